"""Pins of the oracle's right-preconditioned block GMRES(m) (Section 2.1, footnote of 2.2)."""
import numpy as np
import pytest
import scipy.fft
import scipy.sparse.linalg as spla

from synth import config0, tiny_random_job, appendix1
from oracle.assemble import Assembled
from oracle.sparse import to_dense, to_scipy
from oracle.spai import SpaiPattern, spai_build
from oracle.gmres import block_gmres, qr_positive, column_sines, DEP_SINE
from oracle.update import update_pattern
from oracle.pipeline import JobOracle


def _ident(X):
    return X


def test_qr_positive_unique():
    rng = np.random.default_rng(0)
    W = rng.standard_normal((50, 4))
    Q, R = qr_positive(W)
    np.testing.assert_allclose(Q @ R, W, atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(4), atol=1e-14)
    assert np.all(np.diag(R) > 0) and np.allclose(R, np.triu(R))
    # the Cholesky factor of W^T W is the same R (uniqueness of the positive QR)
    np.testing.assert_allclose(R, np.linalg.cholesky(W.T @ W).T, rtol=1e-11)


@pytest.mark.parametrize("seed,k", [(0, 1), (1, 2), (2, 4), (3, 3)])
def test_matches_dense_lu(seed, k):
    job = tiny_random_job(120, 0.04, 30 + seed, k=k)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[0])
    A = to_scipy(job.n, asm.rowptr, asm.col, val)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    pv, _ = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    P = to_scipy(job.n, pat.P_rowptr, pat.P_col, pv)
    X, info = block_gmres(A.__matmul__, P.__matmul__, job.B, m=10, tol=1e-8)
    assert info.converged and not info.breakdown
    Ad = A.toarray()
    X_lu = np.linalg.solve(Ad, job.B)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(X - X_lu) / np.linalg.norm(X_lu) <= 1e-8 * kappa
    assert np.all(np.linalg.norm(job.B - Ad @ X, axis=0) <= 1e-8 * np.linalg.norm(job.B, axis=0))
    # the least-squares residual never increases inside a cycle
    start = 0
    for steps in info.steps:
        h = np.array(info.ls_history[start:start + steps])
        assert np.all(np.diff(h, axis=0) <= 1e-12)
        start += steps


def test_config0_dst_closed_form():
    """C0: A = (1+p) I + 1.01 K is diagonalised by the 2-D DST-I, giving the exact solution."""
    job = config0()
    orc = JobOracle(job)
    p = 0.1
    val, A = orc.A(p)
    pv, _ = orc.spai(val)
    P = orc.P(pv)
    X, info = block_gmres(A.__matmul__, P.__matmul__, job.B, m=30, tol=1e-8)
    assert info.converged
    N = 32
    a = np.arange(1, N + 1)
    lam = (1 + p) + 1.01 * (4 - 2 * np.cos(a[:, None] * np.pi / (N + 1))
                            - 2 * np.cos(a[None, :] * np.pi / (N + 1)))
    X_exact = np.zeros_like(job.B)
    for c in range(job.k):
        b = job.B[:, c].reshape(N, N)  # [y, x]; lam is symmetric in (a, b)
        bh = scipy.fft.dstn(b, type=1)
        X_exact[:, c] = scipy.fft.idstn(bh / lam.T, type=1).ravel()
    kappa = lam.max() / lam.min()
    err = np.linalg.norm(X - X_exact) / np.linalg.norm(X_exact)
    assert err <= 1e-8 * kappa
    assert info.steps[0] <= 30


def test_exact_inverse_preconditioner_one_step():
    job = tiny_random_job(60, 0.08, 41, k=3)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[0])
    A = to_scipy(job.n, asm.rowptr, asm.col, val)
    Ainv = np.linalg.inv(A.toarray())
    X, info = block_gmres(A.__matmul__, lambda V: Ainv @ V, job.B, m=10, tol=1e-10)
    assert info.converged and info.steps == [1]
    np.testing.assert_allclose(X, Ainv @ job.B, rtol=1e-10, atol=1e-12)


def test_finite_termination():
    """No restart and m k >= n: the block Krylov space fills R^n, residual ~ eps."""
    job = tiny_random_job(24, 0.3, 5, k=2)
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[0]))
    X, info = block_gmres(A.__matmul__, _ident, job.B, m=12, tol=1e-13, max_cycles=1)
    assert info.steps[0] <= 12
    assert np.all(info.relres <= 1e-11)


def test_single_rhs_agrees_with_scipy_gmres():
    job = tiny_random_job(150, 0.03, 8, k=1)
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[0]))
    b = job.B[:, 0]
    X, info = block_gmres(A.__matmul__, _ident, job.B, m=30, tol=1e-10)
    x_ref, code = spla.gmres(A, b, restart=30, rtol=1e-12, atol=0.0, maxiter=200)
    assert code == 0 and info.converged
    np.testing.assert_allclose(X[:, 0], x_ref, rtol=1e-7, atol=1e-9 * np.abs(x_ref).max())


def test_appendix1_nonsymmetric():
    """Appendix I (s = 0.5): SPAI on pattern(A) is exact, so one block step; and the
    unpreconditioned solve agrees with the block-diagonal direct solution."""
    job = appendix1(s=0.5)
    orc = JobOracle(job)
    val, A = orc.A(job.p_list[1])
    pv, _ = orc.spai(val)
    X, info = block_gmres(A.__matmul__, orc.P(pv).__matmul__, job.B, m=30, tol=1e-10)
    assert info.converged and info.steps == [1]
    Xd = np.linalg.solve(A.toarray(), job.B)
    np.testing.assert_allclose(X, Xd, rtol=1e-9)
    X2, info2 = block_gmres(A.__matmul__, _ident, job.B, m=30, tol=1e-10, max_cycles=200)
    assert info2.converged
    np.testing.assert_allclose(X2, Xd, rtol=1e-6, atol=1e-8 * np.abs(Xd).max())


def test_zero_rhs_columns():
    job = tiny_random_job(40, 0.1, 12, k=3)
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[0]))
    B = job.B.copy(); B[:, 1] = 0.0
    X, info = block_gmres(A.__matmul__, _ident, B, m=20, tol=1e-10)
    assert info.converged and np.all(X[:, 1] == 0.0)
    np.testing.assert_allclose(A.toarray() @ X, B, atol=1e-8)
    X0, info0 = block_gmres(A.__matmul__, _ident, np.zeros_like(B), m=5)
    assert info0.converged and not X0.any()


def test_fixed_steps_reproduce():
    job = tiny_random_job(80, 0.05, 13, k=2)
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[0]))
    X, info = block_gmres(A.__matmul__, _ident, job.B, m=6, tol=1e-9, max_cycles=50)
    assert info.converged and len(info.steps) > 1  # restarts happened
    X2, _ = block_gmres(A.__matmul__, _ident, job.B, m=6, tol=1e-9, fixed_steps=info.steps)
    np.testing.assert_array_equal(X, X2)


def test_sequence_update_vs_rebuild_config0():
    """Every point of C0 converges to 1e-8 with both policies and they agree."""
    job = config0()
    orc = JobOracle(job)
    upd = orc.run(policy="update")
    reb = orc.run(policy="rebuild")
    for u, r in zip(upd, reb):
        assert u["info"].converged and r["info"].converged
        assert np.all(u["info"].relres <= 1e-8)
        d = np.linalg.norm(u["X"] - r["X"]) / np.linalg.norm(r["X"])
        assert d <= 1e-7


def test_column_sines_brute_force():
    """The sine of each column against the span of the columns before it equals the
    relative residual of its least-squares projection onto them (SVD lstsq)."""
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((40, 5))
    Y[:, 2] = Y[:, 0] - 2.0 * Y[:, 1] + 1e-9 * rng.standard_normal(40)
    Y[:, 3] *= 1e-12  # a tiny but independent column keeps a sine of order one
    Y[:, 4] = Y[:, 3] * 3.0  # an exact multiple of a tiny column
    _, R = qr_positive(Y)
    got = column_sines(Y, R)
    Yn = Y / np.linalg.norm(Y, axis=0)  # the sine does not depend on column scales
    for c in range(5):
        if c == 0:
            want = 1.0
        else:
            coef, *_ = np.linalg.lstsq(Yn[:, :c], Yn[:, c], rcond=None)
            want = np.linalg.norm(Yn[:, c] - Yn[:, :c] @ coef)
        assert abs(got[c] - want) <= 1e-12 + 1e-5 * want, (c, got[c], want)
    assert got[2] < 1e-8 and got[3] > 0.1 and got[4] < 1e-12


def _c0_matrix():
    job = config0()
    orc = JobOracle(job)
    _, A = orc.A(job.p_list[0])
    return job, A


@pytest.mark.parametrize("eps", [0.0, 1e-10, 1e-3])
def test_dependent_rhs_columns(eps):
    """A right-hand side that duplicates another up to eps: the residual block is
    dependent (sine <= 1e-6) for eps = 0 and 1e-10, so the solve stops at the first
    cycle start with X = 0; the verdict agrees with the smallest singular value of
    the column-normalised block (for two unit columns at angle t it is about t/sqrt 2).
    At eps = 1e-3 the block is independent and the solve converges to the LU solution."""
    job, A = _c0_matrix()
    rng = np.random.default_rng(77)
    b = job.B[:, 0]
    B = np.column_stack([b, b + eps * np.linalg.norm(b) * rng.standard_normal(job.n) / np.sqrt(job.n)])
    X, info = block_gmres(A.__matmul__, _ident, B, m=30, tol=1e-8)
    smin = np.linalg.svd(B / np.linalg.norm(B, axis=0), compute_uv=False)[-1]
    dependent = np.sqrt(2.0) * smin <= DEP_SINE
    assert dependent == (eps < 1e-6)
    if dependent:
        assert info.breakdown and info.steps == [0] and not info.converged and not X.any()
    else:
        assert info.converged and not info.breakdown
        X_lu = np.linalg.solve(A.toarray(), B)
        assert np.linalg.norm(X - X_lu) / np.linalg.norm(X_lu) <= 1e-7


def test_rhs_in_invariant_subspace_ends_cycle_then_restarts():
    """b_1 is a combination of two eigenvectors of the symmetric C0 matrix, so its
    Krylov space has dimension 2 (a textbook fact: the grade of b_1 is 2).  Without a
    preconditioner the block Krylov space stops growing at the second block step: the
    first cycle ends there with b_1 solved exactly, and the restart finishes b_2."""
    job, A = _c0_matrix()
    Ad = A.toarray()
    w, U = np.linalg.eigh(Ad)
    b1 = U[:, 3] + 0.5 * U[:, 700]
    B = np.column_stack([b1, job.B[:, 1]])
    X, info = block_gmres(A.__matmul__, _ident, B, m=30, tol=1e-10, max_cycles=10)
    assert info.steps[0] == 2 and len(info.steps) >= 2
    assert info.converged and not info.breakdown
    assert info.ls_history[1][0] <= 1e-13  # b_1 solved within the first cycle
    X_lu = np.linalg.solve(Ad, B)
    assert np.linalg.norm(X - X_lu) / np.linalg.norm(X_lu) <= 1e-9
    # x_1 is the eigen-expansion of b_1
    x1 = U[:, 3] / w[3] + 0.5 * U[:, 700] / w[700]
    assert np.linalg.norm(X[:, 0] - x1) <= 1e-10 * np.linalg.norm(x1)


def test_pipeline_pattern_update_branch():
    """JobOracle.run with the U-pattern update uses Q_l P_1, Q_l column by column the
    dense least squares min ||A(1)e_i - A(l)(:, J_i) q||_2 (SVD lstsq): its X equals
    a block GMRES run with that dense Q_l P_1 for the same block steps, and every
    point converges to the dense LU solution."""
    job = tiny_random_job(48, 0.08, 17, k=2, npts=3)
    orc = JobOracle(job)
    out = orc.run(policy="update", update_kind="pattern", m=10, tol=1e-10)
    n = job.n
    val1, A1 = orc.A(job.p_list[0])
    P1 = orc.P(orc.spai(val1)[0]).toarray()
    pat = orc.pat
    for l, res in enumerate(out):
        vall, Al = orc.A(job.p_list[l])
        Ald, A1d = Al.toarray(), A1.toarray()
        if l == 0:
            Pl = P1
        else:
            Q = np.zeros((n, n))
            for i in range(n):
                J = pat.J_row[pat.J_colptr[i]:pat.J_colptr[i + 1]]
                q, *_ = np.linalg.lstsq(Ald[:, J], A1d[:, i], rcond=None)
                Q[J, i] = q
            Pl = Q @ P1
        Xd, _ = block_gmres(Al.__matmul__, lambda V, Pl=Pl: Pl @ V, job.B, m=10, tol=1e-10,
                            fixed_steps=res["info"].steps)
        assert np.linalg.norm(res["X"] - Xd) <= 1e-11 * np.linalg.norm(Xd), l
        assert res["info"].converged
        X_lu = np.linalg.solve(Ald, job.B)
        assert np.linalg.norm(res["X"] - X_lu) <= 1e-8 * np.linalg.cond(Ald) * np.linalg.norm(X_lu)
