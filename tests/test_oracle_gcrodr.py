"""Pins of the oracle's block GCRO-DR (oracle/gcrodr.py) against facts that do
not come from it: the kr = 0 case is the pinned block GMRES, an exact solution
in the recycled space is found by the projection alone, the harmonic Ritz
values of the first cycle are those of the textbook standard-form formula
(eigenvalues of H_m + H_m^{-T} E_m H_{m+1,m}^T H_{m+1,m} E_m^T), the recycled
basis satisfies Op U = C with orthonormal C, converged solutions match a dense
solve, and the pair rule of the selection on a matrix with known spectrum.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from synth import tiny_random_job
from oracle.assemble import Assembled
from oracle.sparse import to_scipy
from oracle.spai import SpaiPattern, spai_build
from oracle.gmres import block_gmres
from oracle.gcrodr import block_gcrodr, harmonic_select


def _system(seed=31, k=2, n=150, l=0):
    job = tiny_random_job(n, 0.04, seed, k=k)
    asm = Assembled(job)
    val = asm.values(job.s, job.p_list[l])
    A = to_scipy(job.n, asm.rowptr, asm.col, val)
    return job, asm, A


def _jacobi(A):
    d = A.diagonal()
    return lambda X: X / d[:, None] if X.ndim == 2 else X / d


def test_no_recycling_is_block_gmres():
    job, asm, A = _system()
    P = _jacobi(A)
    for steps in ([4, 3], [6]):
        X1, i1 = block_gmres(A.__matmul__, P, job.B, m=10, fixed_steps=steps)
        X2, i2 = block_gcrodr(A.__matmul__, P, job.B, m=10, kr=0, fixed_steps=steps)
        np.testing.assert_array_equal(X1, X2)
        assert i1.steps == i2.steps
    X1, i1 = block_gmres(A.__matmul__, P, job.B, m=8, tol=1e-9)
    X2, i2 = block_gcrodr(A.__matmul__, P, job.B, m=8, kr=0, tol=1e-9)
    np.testing.assert_array_equal(X1, X2)
    assert i1.steps == i2.steps and i2.converged


def test_exact_solution_in_the_recycled_space():
    job, asm, A = _system(k=1)
    P = _jacobi(A)
    Ad = A.toarray()
    b = job.B[:, :1]
    xt = np.linalg.solve(Ad / A.diagonal()[None, :], b)  # Op x~ = b with Op = A D^{-1}
    rec = {"U": np.hstack([xt, np.random.default_rng(1).standard_normal((job.n, 1))])}
    X, info = block_gcrodr(A.__matmul__, P, b, m=10, kr=2, tol=1e-10, recycle=rec)
    assert info.converged and info.steps == []
    np.testing.assert_allclose(X, np.linalg.solve(Ad, b), rtol=1e-9)


def test_first_cycle_harmonic_ritz_values_match_the_standard_formula():
    """Without C the selection solves H_bar^T [I; 0] z = mu H_bar^T H_bar z; for
    k = 1 the harmonic Ritz values theta = 1/mu are the eigenvalues of
    H_m + h^2 H_m^{-T} e_m e_m^T (Morgan's form)."""
    job, asm, A = _system(k=1)
    P = _jacobi(A)
    m = 12
    X, info = block_gmres(A.__matmul__, P, job.B[:, :1], m=m, fixed_steps=[m])
    Hb = info.hessenbergs[0]
    Hm = Hb[:m, :m]
    h = Hb[m, m - 1]
    em = np.zeros(m); em[-1] = 1.0
    theta = np.linalg.eigvals(Hm + h * h * np.linalg.solve(Hm.T, np.outer(em, em)))
    WtV = np.vstack([np.eye(m), np.zeros((1, m))])
    for kr in (1, 3, 5):
        Pk, mu = harmonic_select(Hb, WtV, kr)
        want = np.sort(np.abs(theta))[:Pk.shape[1]]
        np.testing.assert_allclose(np.sort(np.abs(1.0 / mu)), want, rtol=1e-8)
        # each column pair / column spans eigenvectors of the generalized problem
        M = np.linalg.solve(Hb.T @ Hb, Hb.T @ WtV)
        res = M @ Pk - Pk @ np.linalg.lstsq(Pk, M @ Pk, rcond=None)[0]
        assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(M) * np.linalg.norm(Pk)


def test_pair_rule_on_a_known_spectrum():
    """G = I and WtV with eigenvalues 3, 2 +- 1.5i, 1: |mu| = 3, 2.5, 2.5, 1."""
    T = np.zeros((5, 5))
    T[0, 0] = 3.0
    T[1:3, 1:3] = [[2.0, -1.5], [1.5, 2.0]]
    T[3, 3] = 1.0
    T[4, 4] = 0.5
    Qr, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((5, 5)))
    WtV = Qr @ T @ Qr.T
    G = np.eye(5)
    for kr, dims in ((1, 1), (2, 1), (3, 3), (4, 4)):
        Pk, mu = harmonic_select(G, WtV, kr)
        assert Pk.shape[1] == dims, kr
        # the span is the invariant subspace of the selected eigenvalues
        want = Qr[:, :dims]
        s = sla.subspace_angles(Pk, want)
        assert s.max() < 1e-10


def test_recycled_basis_and_dense_solution():
    job, asm, A = _system(k=2)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    val = asm.values(job.s, job.p_list[0])
    pv, _ = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    Pm = to_scipy(job.n, pat.P_rowptr, pat.P_col, pv)
    rec = {}
    X, info = block_gcrodr(A.__matmul__, Pm.__matmul__, job.B, m=5, kr=4, tol=1e-10, recycle=rec)
    assert info.converged and len(info.steps) >= 2
    Ad = A.toarray()
    Xd = np.linalg.solve(Ad, job.B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) <= 1e-10 * np.linalg.cond(Ad)
    U = rec["U"]
    kc = U.shape[1]
    assert U.shape[0] == job.n and kc in (3, 4)  # a conjugate pair may not fit
    C = A @ (Pm @ U)
    np.testing.assert_allclose(C.T @ C, np.eye(kc), atol=1e-9)


def test_recycling_across_a_sequence_saves_steps():
    """Nearby systems of one job: the recycled space from the earlier points
    lowers the block steps the later points need (m small so that restarts
    happen and the deflation matters)."""
    job = tiny_random_job(150, 0.04, 33, k=2)
    asm = Assembled(job)
    rec = {}
    plain, recycled = 0, 0
    for l in range(len(job.p_list)):
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[l]))
        P = _jacobi(A)
        _, i0 = block_gmres(A.__matmul__, P, job.B, m=4, tol=1e-10, max_cycles=60)
        _, i1 = block_gcrodr(A.__matmul__, P, job.B, m=4, kr=6, tol=1e-10, max_cycles=60, recycle=rec)
        assert i0.converged and i1.converged
        plain += sum(i0.steps)
        recycled += sum(i1.steps)
    assert recycled < plain
