"""Pins of the oracle's assembly of A(s,p) = s^2 M(p) + s D(p) + K(p) (Section 1.1)."""
import numpy as np
import pytest

from synth import config0, tiny_random_job, appendix1, gyro_like_job, gyro_coefs
from oracle.assemble import Assembled, affine_values, union_pattern
from oracle.sparse import to_dense, check_csr
from oracle.diagnostics import fro_I_minus_A, fro_diff


def _dense_terms(job):
    return {r: to_dense(job.n, T.rowptr, T.col, T.val) for r, T in job.terms.items()}


@pytest.mark.parametrize("seed", range(6))
def test_union_pattern_brute_force(seed):
    job = tiny_random_job(13 + seed, 0.15, seed)
    asm = Assembled(job)
    check_csr(job.n, asm.rowptr, asm.col)
    mask = np.eye(job.n, dtype=bool)
    for T in job.terms.values():
        D = np.zeros((job.n, job.n), dtype=bool)
        for i in range(job.n):
            D[i, T.col[T.rowptr[i]:T.rowptr[i + 1]]] = True
        mask |= D
    rr, cc = np.nonzero(mask)  # row-major order == CSR order
    np.testing.assert_array_equal(asm.col, cc)
    np.testing.assert_array_equal(np.diff(asm.rowptr), np.bincount(rr, minlength=job.n))
    # slot maps point at the right term entries
    rows = np.repeat(np.arange(job.n), np.diff(asm.rowptr))
    dense = _dense_terms(job)
    for role, m in asm.maps.items():
        T = job.terms[role]
        got = np.where(m >= 0, T.val[np.maximum(m, 0)], 0.0)
        np.testing.assert_array_equal(got, dense[role][rows, asm.col])
        assert np.count_nonzero(m >= 0) == T.nnz


def test_laplace_transform_semantics():
    """A(s,p) v is what M(p) x'' + D(p) x' + K(p) x gives for x(t) = exp(s t) v.

    The derivatives of x at t = 0 are taken by central differences, so this pins
    the roles of s^2 and s without restating the assembly formula.
    """
    job = tiny_random_job(17, 0.2, 3, roles=("M0", "M1", "D0", "D1", "K0", "K1"))
    asm = Assembled(job)
    dense = _dense_terms(job)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(job.n)
    for s, p in ((0.7, 0.3), (1.9, -0.4), (-0.6, 1.3)):
        Mp = dense["M0"] + p * dense["M1"]
        Dp = dense["D0"] + p * dense["D1"]
        Kp = dense["K0"] + p * dense["K1"]
        h = 1e-3
        x = lambda t: np.exp(s * t) * v  # noqa: E731
        xdd = (x(h) - 2 * x(0.0) + x(-h)) / (h * h)
        xd = (x(h) - x(-h)) / (2 * h)
        ode = Mp @ xdd + Dp @ xd + Kp @ x(0.0)
        A = to_dense(job.n, asm.rowptr, asm.col, asm.values(s, p))
        np.testing.assert_allclose(A @ v, ode, rtol=1e-5, atol=1e-5 * np.abs(ode).max())


def test_config0_closed_forms():
    """C0: A(p) = (1+p) I + 1.01 K with K the 2-D Dirichlet 5-point Laplacian."""
    job = config0()
    asm = Assembled(job)
    assert asm.nnz == 4992
    v1 = asm.values(job.s, 0.1)
    for p in job.p_list:
        v = asm.values(job.s, p)
        # ||A(l) - A(1)||_F = |p_l - p_1| s ||M||_F = |dp| * 32  (analogue of Table 2, column 4)
        assert fro_diff(v1, v) == pytest.approx(abs(p - 0.1) * 32.0, rel=1e-13)
        # ||I - A(l)||_F = sqrt(1024 (p + 4.04)^2 + 3968 * 1.01^2)   (Table 2, column 3)
        want = np.sqrt(1024 * (p + 4.04) ** 2 + 3968 * 1.01 ** 2)
        assert fro_I_minus_A(job.n, asm.rowptr, asm.col, v) == pytest.approx(want, rel=1e-13)
    # spectrum: eigenvalues of the 2-D Laplacian are 4 - 2cos(a pi/33) - 2cos(b pi/33)
    A = to_dense(job.n, asm.rowptr, asm.col, asm.values(1.0, 0.3))
    a = np.arange(1, 33)
    lam = (4 - 2 * np.cos(a[:, None] * np.pi / 33) - 2 * np.cos(a[None, :] * np.pi / 33)).ravel()
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(1.3 + 1.01 * lam), rtol=1e-12)


def test_appendix1_difference_confined():
    """Appendix I: A(s,p_j) - A(s,p_1) is nonzero only in the leading 2x2 block."""
    job = appendix1(s=0.5)
    asm = Assembled(job)
    v1 = asm.values(0.5, job.p_list[0])
    for p in job.p_list[1:]:
        d = asm.values(0.5, p) - v1
        rows = np.repeat(np.arange(job.n), np.diff(asm.rowptr))
        nz = np.nonzero(d)[0]
        assert set(zip(rows[nz], asm.col[nz])) == {(0, 1), (1, 0)}
        np.testing.assert_allclose(np.abs(d[nz]), abs(p - job.p_list[0]), rtol=1e-14)


def test_affine_union_pattern_brute_force():
    """The union pattern of a list of terms (the affine form) against dense masks,
    and every slot map against the dense term values."""
    job = gyro_like_job(dims=(6, 5, 4))
    asm = Assembled(job)
    check_csr(job.n, asm.rowptr, asm.col)
    mask = np.eye(job.n, dtype=bool)
    dense = [to_dense(job.n, T.rowptr, T.col, T.val) for T in job.aterms]
    for T in job.aterms:
        for i in range(job.n):
            mask[i, T.col[T.rowptr[i]:T.rowptr[i + 1]]] = True
    rr, cc = np.nonzero(mask)
    np.testing.assert_array_equal(asm.col, cc)
    np.testing.assert_array_equal(np.diff(asm.rowptr), np.bincount(rr, minlength=job.n))
    rows = np.repeat(np.arange(job.n), np.diff(asm.rowptr))
    for t, T in enumerate(job.aterms):
        m = asm.maps[t]
        got = np.where(m >= 0, T.val[np.maximum(m, 0)], 0.0)
        np.testing.assert_array_equal(got, dense[t][rows, asm.col])
        assert np.count_nonzero(m >= 0) == T.nnz
    # the long-range term widens the union beyond the 7-point stencil
    assert asm.nnz > job.aterms[0].nnz


def test_affine_gyroscope_semantics():
    """The gyroscope model of Section 3: s^2 M(d) x + s D(theta, d) x + K(d) x with
    M(d) = M1 + d M2, D = theta (D1 + d D2), K(d) = K1 + (1/d) K2 + d K3 (alpha = beta
    = 0).  For x(t) = exp(s t) v, the affine assembly at the point's seven
    coefficients times v equals M(d) x'' + D x' + K(d) x at t = 0, the derivatives
    taken by central differences: this pins each coefficient (s^2, s^2 d, s theta,
    s theta d, 1/d, d) to its term without restating the coefficient list."""
    job = gyro_like_job(dims=(6, 5, 4))
    asm = Assembled(job)
    mats = {name: to_dense(job.n, T.rowptr, T.col, T.val) for name, T in job.meta["matrices"].items()}
    rng = np.random.default_rng(8)
    v = rng.standard_normal(job.n)
    for s, theta, d in ((0.8, 0.4, 1.3), (-1.1, 0.7, 0.6), (1.6, -0.2, 2.0)):
        Md = mats["M1"] + d * mats["M2"]
        Dd = theta * (mats["D1"] + d * mats["D2"])
        Kd = mats["K1"] + (1.0 / d) * mats["K2"] + d * mats["K3"]
        h = 1e-3
        x = lambda t: np.exp(s * t) * v  # noqa: E731
        xdd = (x(h) - 2 * x(0.0) + x(-h)) / (h * h)
        xd = (x(h) - x(-h)) / (2 * h)
        ode = Md @ xdd + Dd @ xd + Kd @ x(0.0)
        A = to_dense(job.n, asm.rowptr, asm.col, asm.values_c(gyro_coefs(s, theta, d)))
        np.testing.assert_allclose(A @ v, ode, rtol=1e-5, atol=1e-5 * np.abs(ode).max())


def test_roles_as_an_affine_list():
    """A job of roles written as a term list with the role coefficients
    (s^2, s^2 p, s, s p, 1, p) assembles to the same values as by roles."""
    job = tiny_random_job(21, 0.15, 4, roles=("M0", "M1", "D0", "D1", "K0", "K1"))
    asm = Assembled(job)
    terms = [job.terms[r] for r in ("M0", "M1", "D0", "D1", "K0", "K1")]
    rp, ci, maps = union_pattern(job.n, terms)
    np.testing.assert_array_equal(rp, asm.rowptr)
    np.testing.assert_array_equal(ci, asm.col)
    for s, p in ((0.7, 0.3), (1.9, -0.4)):
        c = [s * s, s * s * p, s, s * p, 1.0, p]
        np.testing.assert_allclose(affine_values(terms, maps, asm.nnz, c), asm.values(s, p), rtol=1e-14,
                                   atol=1e-14 * np.abs(asm.values(s, p)).max())
