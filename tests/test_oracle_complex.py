"""Pins of the complex-point oracle (oracle/complexsys.py and block GMRES on
complex blocks) against facts that do not come from the oracle itself: the
real case (where it must reduce to the pinned real routines), closed forms,
optimality conditions of the least squares, a dense complex solve, and the
real-form identities R(A) R(x) = R(A x) and R(i x) = J R(x).
"""
import numpy as np
import pytest

from synth import gyro_complex_job
from oracle.complexsys import (ComplexAssembled, matvec, real_form_csr, real_form, complex_of, spai_complex,
                               spai_complex_column, diag_factors_complex, update_diag_complex, to_dense)
from oracle.spai import SpaiPattern, spai_build, solve_column
from oracle.update import diag_factors
from oracle.gmres import block_gmres

pytestmark = pytest.mark.filterwarnings("ignore::numpy.exceptions.ComplexWarning")


@pytest.fixture(scope="module")
def job():
    return gyro_complex_job(dims=(4, 3, 3), k=2)


@pytest.fixture(scope="module")
def asm(job):
    return ComplexAssembled(job)


def test_real_form_matvec_and_rotation(job, asm):
    rng = np.random.default_rng(7)
    v = asm.values(job.coefs[1])
    assert np.iscomplexobj(v) and np.abs(v.imag).max() > 0.1
    rp2, c2, v2 = real_form_csr(job.n, asm.rowptr, asm.col, v)
    x = rng.standard_normal((job.n, 3)) + 1j * rng.standard_normal((job.n, 3))
    # R(A) R(x) = R(A x), with A x from a dense complex product
    Ad = to_dense(job.n, asm.rowptr, asm.col, v)
    np.testing.assert_allclose(matvec(2 * job.n, rp2, c2, v2, real_form(x)), real_form(Ad @ x), rtol=0, atol=1e-12)
    # multiplication by sqrt(-1) is the rotation (x_re, x_im) -> (-x_im, x_re)
    r = real_form(1j * x)
    np.testing.assert_array_equal(r[0::2], -real_form(x)[1::2])
    np.testing.assert_array_equal(r[1::2], real_form(x)[0::2])
    np.testing.assert_array_equal(complex_of(real_form(x)), x)
    # whole 2x2 blocks: rows 2i, 2i+1 hold the same columns, in pairs
    for i in range(job.n):
        a, b, c = rp2[2 * i], rp2[2 * i + 1], rp2[2 * i + 2]
        np.testing.assert_array_equal(c2[a:b], c2[b:c])
        assert np.all(c2[a:b:2] % 2 == 0) and np.all(c2[a + 1:b:2] == c2[a:b:2] + 1)


def test_complex_values_are_the_coefficient_sum(job, asm):
    """Each stored value is sum_t c_t T_t(i, j), read from the terms by brute force."""
    c = job.coefs[2]
    v = asm.values(c)
    for e in range(0, asm.nnz, 7):
        i = int(np.searchsorted(asm.rowptr, e, side="right") - 1)
        j = int(asm.col[e])
        want = 0j
        for t, T in enumerate(job.aterms):
            for f in range(T.rowptr[i], T.rowptr[i + 1]):
                if T.col[f] == j:
                    want += c[t] * T.val[f]
        assert v[e] == pytest.approx(want, abs=1e-14)


def test_spai_complex_reduces_to_real_oracle(job, asm):
    """With real coefficients the complex SPAI is the (pinned) real SPAI."""
    c = np.real(job.coefs[0]).astype(complex)
    c[3:5] = 0.0  # no damping: a real matrix
    v = asm.values(c)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    cols = list(range(0, job.n, 5))
    pc, rc = spai_complex(job.n, asm.rowptr, asm.col, v, pat, cols)
    pr, rr = spai_build(job.n, asm.rowptr, asm.col, v.real, pat, cols)
    m = ~np.isnan(pr)
    np.testing.assert_allclose(pc[m].real, pr[m], rtol=1e-10, atol=1e-13)
    assert np.abs(pc[m].imag).max() < 1e-13
    np.testing.assert_allclose(rc[cols], rr[cols], rtol=1e-9, atol=1e-14)


def test_spai_complex_column_optimality(job, asm):
    """The complex least-squares residual is orthogonal (Hermitian product) to the
    columns of A(I_j, J_j), and no nearby p does better."""
    v = asm.values(job.coefs[1])
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    rng = np.random.default_rng(3)
    A = to_dense(job.n, asm.rowptr, asm.col, v)
    for j in (0, 7, 19, job.n - 1):
        p, rho = spai_complex_column(job.n, asm.rowptr, asm.col, v, pat, j)
        I, J = pat.I(j), pat.J(j)
        Ahat = A[np.ix_(I, J)]
        r = (I == j).astype(complex) - Ahat @ p
        assert np.abs(Ahat.conj().T @ r).max() < 1e-12
        # the full column residual equals the local one (rows outside I_j are zero)
        full = np.zeros(job.n, dtype=complex)
        full[J] = p
        e = np.zeros(job.n); e[j] = 1.0
        assert np.linalg.norm(e - A @ full) == pytest.approx(rho, rel=1e-10)
        for _ in range(3):
            d = 1e-3 * (rng.standard_normal(p.size) + 1j * rng.standard_normal(p.size))
            assert np.linalg.norm((I == j) - Ahat @ (p + d)) > rho


def test_real_form_spai_columns_are_the_complex_column(job, asm):
    """On the real form (whole 2x2 blocks), the real SPAI columns 2j and 2j+1
    (the pinned real Householder oracle) are R(p_j) and R(i p_j)."""
    v = asm.values(job.coefs[3])
    rp2, c2, v2 = real_form_csr(job.n, asm.rowptr, asm.col, v)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    pat2 = SpaiPattern(2 * job.n, rp2, c2)
    for j in (1, 11, 30):
        p, rho = spai_complex_column(job.n, asm.rowptr, asm.col, v, pat, j)
        J = pat.J(j)
        for part, z in ((0, p), (1, 1j * p)):
            x, r = solve_column(2 * job.n, rp2, c2, v2, pat2, 2 * j + part)
            J2 = pat2.J(2 * j + part)
            np.testing.assert_array_equal(J2[0::2], 2 * J)
            np.testing.assert_allclose(x, real_form(z), rtol=0, atol=1e-11 * np.abs(p).max())
            assert r == pytest.approx(rho, rel=1e-9)


def test_complex_diag_factors(job, asm):
    v1 = asm.values(job.coefs[0])
    # A(l) = gamma A(1): q = 1 / gamma exactly up to rounding, zero residuals
    g = 0.7 - 1.3j
    q, rho = diag_factors_complex(job.n, asm.rowptr, asm.col, v1, g * v1)
    np.testing.assert_allclose(q, np.full(job.n, 1.0 / g), rtol=1e-13)
    assert rho.max() < 1e-12
    # real data: the pinned real factors
    vr = asm.values(np.real(job.coefs[0]))
    vr2 = asm.values(np.real(job.coefs[1]))
    q, _ = diag_factors_complex(job.n, asm.rowptr, asm.col, vr, vr2)
    np.testing.assert_allclose(q.real, diag_factors(job.n, asm.rowptr, asm.col, vr.real, vr2.real), rtol=1e-14)
    assert np.abs(q.imag).max() == 0.0
    # optimality: a_l^H (a_1 - q a_l) = 0 per column, and rho is that residual
    vl = asm.values(job.coefs[2])
    q, rho = diag_factors_complex(job.n, asm.rowptr, asm.col, v1, vl)
    A1 = to_dense(job.n, asm.rowptr, asm.col, v1)
    Al = to_dense(job.n, asm.rowptr, asm.col, vl)
    for i in range(0, job.n, 5):
        r = A1[:, i] - q[i] * Al[:, i]
        assert abs(np.vdot(Al[:, i], r)) < 1e-12 * np.linalg.norm(Al[:, i]) * np.linalg.norm(A1[:, i])
        assert np.linalg.norm(r) == pytest.approx(rho[i], rel=1e-12)
    # P_l = diag(q) P_1 row by row
    P1 = np.arange(1, asm.nnz + 1) * (1 + 0.5j)
    Pl = update_diag_complex(job.n, asm.rowptr, P1, q)
    i = 4
    np.testing.assert_allclose(Pl[asm.rowptr[i]:asm.rowptr[i + 1]], q[i] * P1[asm.rowptr[i]:asm.rowptr[i + 1]],
                               rtol=1e-15)


def _operators(job, asm, l):
    v = asm.values(job.coefs[l])
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    pv, _ = spai_complex(job.n, asm.rowptr, asm.col, v, pat)
    A = lambda X: matvec(job.n, asm.rowptr, asm.col, v, X)  # noqa: E731
    P = lambda X: matvec(job.n, pat.P_rowptr, pat.P_col, pv, X)  # noqa: E731
    return v, pat, pv, A, P


def test_complex_block_gmres_solves_the_dense_system(job, asm):
    v, pat, pv, A, P = _operators(job, asm, 1)
    X, info = block_gmres(A, P, job.B, m=30, tol=1e-10)
    assert info.converged and X.dtype == np.complex128
    Xd = np.linalg.solve(to_dense(job.n, asm.rowptr, asm.col, v), job.B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 1e-8


def test_real_form_block_gmres_with_rotated_block_is_complex_block_gmres(job, asm):
    """Block GMRES on the real form with [R(B), R(iB)] spans the real form of the
    complex block Krylov space of B: its first k columns are R(X) of complex
    block GMRES, step for step, and the other k are R(i X)."""
    v, pat, pv, A, P = _operators(job, asm, 2)
    rp2, c2, v2 = real_form_csr(job.n, asm.rowptr, asm.col, v)
    prp, pc2, pv2 = real_form_csr(job.n, pat.P_rowptr, pat.P_col, pv)
    A2 = lambda X: matvec(2 * job.n, rp2, c2, v2, X)  # noqa: E731
    P2 = lambda X: matvec(2 * job.n, prp, pc2, pv2, X)  # noqa: E731
    k = job.k
    for steps in ([2], [5, 3]):
        Xc, ic = block_gmres(A, P, job.B, m=30, fixed_steps=steps)
        Br = np.hstack([real_form(job.B), real_form(1j * job.B)])
        Xr, ir = block_gmres(A2, P2, Br, m=30, fixed_steps=steps)
        np.testing.assert_allclose(Xr[:, :k], real_form(Xc), rtol=0, atol=1e-10 * np.abs(Xc).max())
        np.testing.assert_allclose(Xr[:, k:], real_form(1j * Xc), rtol=0, atol=1e-10 * np.abs(Xc).max())
        for a, b in zip(ic.ls_history, ir.ls_history):
            np.testing.assert_allclose(b[:k], a, rtol=1e-8)
            np.testing.assert_allclose(b[k:], a, rtol=1e-8)
