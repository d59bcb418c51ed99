"""The library's host-side harmonic Ritz choice of block GCRO-DR
(pmor_harmonic_ritz: Cholesky reduction, Hessenberg form, complex Schur form
by the shifted QR iteration, eigenvectors by back substitution) against the
oracle's choice (library generalized eigensolver): the same eigenvalues and the
same chosen subspace on random matrices of many sizes, the pair rule on a
known spectrum, and the error for a rank-deficient G.  Runs on the CPU."""
import ctypes as C

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.gcrodr import harmonic_select


def _host(G, WtV, kr):
    from paper_1809_06574_amd import lib as L
    rows, N = G.shape
    Pk = np.zeros((N, max(kr, 1)))
    mr = np.zeros(max(kr, 1))
    mi = np.zeros(max(kr, 1))
    cnt = C.c_int32()
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    G = np.ascontiguousarray(G, dtype=np.float64)
    W = np.ascontiguousarray(WtV, dtype=np.float64)
    rc = L.pmor_harmonic_ritz(rows, N, dp(G), dp(W), kr, dp(Pk), dp(mr), dp(mi), C.byref(cnt))
    return rc, Pk[:, :cnt.value], mr[:cnt.value] + 1j * mi[:cnt.value]


@pytest.mark.parametrize("seed", range(6))
def test_matches_the_oracle_choice(seed):
    rng = np.random.default_rng(seed)
    for _ in range(8):
        N = int(rng.integers(2, 60))
        rows = N + int(rng.integers(0, 6))
        G = rng.standard_normal((rows, N))
        W = rng.standard_normal((rows, N))
        for kr in (1, 2, 5, 8, 16):
            rc, P2, m2 = _host(G, W, kr)
            assert rc == 0
            P1, m1 = harmonic_select(G, W, kr)
            assert P1.shape == P2.shape
            if P1.shape[1]:
                assert sla.subspace_angles(P1, P2).max() < 1e-8
                for x in m1:
                    assert np.min(np.abs(m2 - x)) <= 1e-9 * np.abs(m1).max()


def test_block_hessenberg_shape_of_a_gmres_cycle():
    """G = Hbar (block upper Hessenberg, k = 4, 6 steps) and WtV = [I; 0], as in
    a first cycle."""
    rng = np.random.default_rng(11)
    k, j = 4, 6
    Hb = np.zeros(((j + 1) * k, j * k))
    for c in range(j):
        Hb[: (c + 1) * k, c * k:(c + 1) * k] = rng.standard_normal(((c + 1) * k, k))
        Hb[(c + 1) * k:(c + 2) * k, c * k:(c + 1) * k] = np.triu(rng.standard_normal((k, k))) + 3 * np.eye(k)
    W = np.vstack([np.eye(j * k), np.zeros((k, j * k))])
    for kr in (4, 8, 16):
        rc, P2, m2 = _host(Hb, W, kr)
        P1, m1 = harmonic_select(Hb, W, kr)
        assert rc == 0 and P1.shape == P2.shape
        assert sla.subspace_angles(P1, P2).max() < 1e-8


def test_pair_rule_and_rank_deficient_G():
    T = np.zeros((5, 5))
    T[0, 0] = 3.0
    T[1:3, 1:3] = [[2.0, -1.5], [1.5, 2.0]]
    T[3, 3] = 1.0
    T[4, 4] = 0.5
    Qr, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((5, 5)))
    W = Qr @ T @ Qr.T
    for kr, dims in ((1, 1), (2, 1), (3, 3), (4, 4)):
        rc, Pk, mu = _host(np.eye(5), W, kr)
        assert rc == 0 and Pk.shape[1] == dims
        assert sla.subspace_angles(Pk, Qr[:, :dims]).max() < 1e-10
    G = np.zeros((5, 5))
    G[:, :4] = np.random.default_rng(5).standard_normal((5, 4))
    from paper_1809_06574_amd import lib as L
    rc, _, _ = _host(G, W, 2)
    assert rc == L.PMOR_ESINGULAR
