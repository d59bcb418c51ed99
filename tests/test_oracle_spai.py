"""Pins of the oracle's SPAI (Section 2.2): patterns, Householder LS, closed forms."""
import numpy as np
import pytest

from synth import config0, tiny_random_job, appendix1
from synth.gen import CSR, diagonal
from oracle.assemble import Assembled
from oracle.sparse import to_dense, to_scipy
from oracle.spai import (SpaiPattern, householder, householder_lstsq, spai_build,
                         SingularColumn, pattern_of_A)
from oracle.diagnostics import fro_from_residuals


def _dense_P(pat, pv):
    n = pat.n
    return to_dense(n, pat.P_rowptr, pat.P_col, pv)


def _structural(n, rowptr, col):
    S = np.zeros((n, n), dtype=bool)
    for i in range(n):
        S[i, col[rowptr[i]:rowptr[i + 1]]] = True
    return S


@pytest.mark.parametrize("seed", range(5))
def test_pattern_and_shadow_brute_force(seed):
    job = tiny_random_job(15 + 2 * seed, 0.12, seed)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    S = _structural(job.n, asm.rowptr, asm.col)
    for j in range(job.n):
        J = np.nonzero(S[:, j] | (np.arange(job.n) == j))[0]
        np.testing.assert_array_equal(pat.J(j), J)
        I = np.nonzero(S[:, J].any(axis=1))[0]
        np.testing.assert_array_equal(pat.I(j), I)
    # CSR of P is the transpose of the J sets, and the slot map is consistent
    for j in range(job.n):
        for t, i in enumerate(pat.J(j)):
            slot = pat.P_slot[pat.J_colptr[j] + t]
            assert pat.P_col[slot] == j
            assert pat.P_rowptr[i] <= slot < pat.P_rowptr[i + 1]


def test_householder_reflector():
    rng = np.random.default_rng(1)
    for x in (rng.standard_normal(7), -np.abs(rng.standard_normal(5)), np.array([0.0, 3.0, 4.0]),
              np.array([2.0, 0.0, 0.0])):
        v, tau, beta = householder(x)
        H = np.eye(x.size) - tau * np.outer(v, v)
        np.testing.assert_allclose(H @ x, beta * np.eye(x.size)[0], atol=1e-14 * np.linalg.norm(x))
        np.testing.assert_allclose(H @ H.T, np.eye(x.size), atol=1e-14)
        assert abs(beta) == pytest.approx(np.linalg.norm(x), rel=1e-15)
        if np.any(x[1:] != 0):
            assert np.sign(beta) == (-1.0 if x[0] >= 0 else 1.0)  # larfg: beta = -sign(x0)||x||


@pytest.mark.parametrize("shape,cond", [((25, 7), 1e1), ((40, 40), 1e3), ((129, 40), 1e6), ((9, 1), 1.0)])
def test_lstsq_matches_svd_solver(shape, cond):
    rng = np.random.default_rng(shape[0])
    m, k = shape
    U, _ = np.linalg.qr(rng.standard_normal((m, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    A = U @ np.diag(np.geomspace(1.0, 1.0 / cond, k)) @ V.T
    b = rng.standard_normal(m)
    x, rho = householder_lstsq(A, b)
    x_ref, *_ = np.linalg.lstsq(A, b, rcond=None)  # SVD-based
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-12 * cond * np.linalg.norm(x_ref))
    assert rho == pytest.approx(np.linalg.norm(b - A @ x_ref), rel=1e-9, abs=1e-14 * cond * np.linalg.norm(b))
    # normal-equations (KKT) residual
    assert np.linalg.norm(A.T @ (b - A @ x)) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(b) * cond


@pytest.mark.parametrize("seed", range(4))
def test_columns_match_full_lstsq(seed):
    """Each SPAI column equals the SVD least-squares solution on the *full* column block."""
    job = tiny_random_job(20 + seed, 0.15, 10 + seed)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[0])
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    pv, rho = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    A = to_dense(job.n, asm.rowptr, asm.col, val)
    P = _dense_P(pat, pv)
    for j in range(job.n):
        J = pat.J(j)
        e = np.zeros(job.n); e[j] = 1.0
        x_ref, *_ = np.linalg.lstsq(A[:, J], e, rcond=None)
        np.testing.assert_allclose(P[J, j], x_ref, rtol=1e-11, atol=1e-13)
        assert rho[j] == pytest.approx(np.linalg.norm(e - A[:, J] @ x_ref), rel=1e-9, abs=1e-14)
        mask = np.ones(job.n, dtype=bool); mask[J] = False
        assert not np.any(P[mask, j])
    # Frobenius identity of Section 2.2: ||I - A P||_F^2 = sum_j rho_j^2
    assert np.linalg.norm(np.eye(job.n) - A @ P) == pytest.approx(fro_from_residuals(rho), rel=1e-12)


def test_full_pattern_gives_inverse():
    job = tiny_random_job(24, 0.2, 77)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[1])
    n = job.n
    full = (np.arange(n + 1, dtype=np.int32) * n, np.tile(np.arange(n, dtype=np.int32), n))
    pat = SpaiPattern(n, asm.rowptr, asm.col, explicit=full)
    pv, rho = spai_build(n, asm.rowptr, asm.col, val, pat)
    A = to_dense(n, asm.rowptr, asm.col, val)
    Ainv = np.linalg.inv(A)
    kappa = np.linalg.cond(A)
    np.testing.assert_allclose(_dense_P(pat, pv), Ainv, atol=1e-13 * kappa * np.abs(Ainv).max())
    assert np.all(rho <= 1e-12 * kappa)


def test_diagonal_matrix_and_diagonal_pattern():
    rng = np.random.default_rng(3)
    d = rng.uniform(0.5, 3.0, 30) * np.where(rng.random(30) < 0.5, -1, 1)
    D = diagonal(d)
    pat = SpaiPattern(30, D.rowptr, D.col)
    pv, rho = spai_build(30, D.rowptr, D.col, D.val, pat)
    np.testing.assert_allclose(_dense_P(pat, pv), np.diag(1.0 / d), rtol=1e-15)
    assert np.all(rho <= 1e-15)
    # a diagonal pattern on a general matrix: p_jj = a_jj / ||A e_j||^2
    job = tiny_random_job(19, 0.25, 4)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[0])
    n = job.n
    dpat = SpaiPattern(n, asm.rowptr, asm.col,
                       explicit=(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)))
    pv, _ = spai_build(n, asm.rowptr, asm.col, val, dpat)
    A = to_dense(n, asm.rowptr, asm.col, val)
    np.testing.assert_allclose(pv, np.diag(A) / np.sum(A * A, axis=0), rtol=1e-13)


def test_appendix1_exact_block_inverses():
    """Appendix I at s = 0.5: A is block diagonal, so SPAI on pattern(A) is the exact inverse."""
    s = 0.5
    job = appendix1(s=s)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    for p in job.p_list:
        pv, rho = spai_build(job.n, asm.rowptr, asm.col, asm.values(s, p), pat)
        P = to_scipy(job.n, pat.P_rowptr, pat.P_col, pv).toarray()
        lead = np.array([[s + 1, p], [-p, s + 1]]) / ((s + 1) ** 2 + p ** 2)
        np.testing.assert_allclose(P[0:2, 0:2], lead, rtol=1e-14)
        for b, w in ((2, 200.0), (4, 400.0)):
            blk = np.array([[s + 1, w], [-w, s + 1]]) / ((s + 1) ** 2 + w ** 2)
            np.testing.assert_allclose(P[b:b + 2, b:b + 2], blk, rtol=1e-13)
        np.testing.assert_allclose(np.diag(P)[6:], 1.0 / (s - np.arange(1, 1001)), rtol=1e-14)
        assert np.all(rho <= 1e-14)


def test_singular_column_reported():
    job = tiny_random_job(12, 0.2, 9)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[0]).copy()
    # zero out column 5 of A: the local least-squares problem of any column whose
    # pattern contains 5 becomes rank deficient
    val[asm.col == 5] = 0.0
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    with pytest.raises(SingularColumn) as exc:
        spai_build(job.n, asm.rowptr, asm.col, val, pat, columns=[5])
    assert exc.value.column == 5


def test_config0_spai_quality():
    """C0 with SPAI on pattern(A): the columns equal the full-block SVD solution (sample)."""
    job = config0()
    asm = Assembled(job)
    val = asm.values(1.0, 0.1)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    cols = [0, 1, 31, 32, 33, 500, 1023]
    pv, rho = spai_build(job.n, asm.rowptr, asm.col, val, pat, columns=cols)
    A = to_dense(job.n, asm.rowptr, asm.col, val)
    P = _dense_P(pat, np.nan_to_num(pv))
    for j in cols:
        J = pat.J(j)
        e = np.zeros(job.n); e[j] = 1.0
        x_ref, *_ = np.linalg.lstsq(A[:, J], e, rcond=None)
        np.testing.assert_allclose(P[J, j], x_ref, rtol=1e-12)
    assert pat.J(500).size == 5 and pat.I(500).size == 13  # interior 5-point column
