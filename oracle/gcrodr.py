"""Block GCRO-DR: block GMRES with a recycled subspace — test infrastructure.

The paper solves its sequences with block GCRO and recycling (Section 3, the
solver of Table 5): a subspace found while solving one system is kept and
reused for the next ones, which is where the method pays off across the
points of a parametric sequence.  The steps below are those of GCRO with
deflated restarting (harmonic Ritz vectors as the recycled space), for a block
of right-hand sides and right preconditioning (Op = A P, X = P X~):

Carried between calls: U~ (n x kc), a basis of the recycled space.

1. Entering a system with U~: C = Op U~, thin QR C = Q R (positive diagonal),
   C <- Q, U <- U~ R^{-1}, so that Op U = C and C has orthonormal columns.
2. Each cycle starts from the true residual R = B - A X and, with C, projects
   it: T = C^T R, X <- X + P U T, R <- R - C T (the best correction in
   span(U); afterwards R is orthogonal to C).
3. Stop if every column has ||r_c|| <= tol ||b_c||; block QR R = V_1 S (the
   dependent-column test of ``oracle.gmres``).
4. Block Arnoldi on (I - C C^T) Op: for j = 1..m, W = Op V_j, two classical
   Gram-Schmidt passes against [C, V_1..V_j] (the C coefficients accumulate in
   B_j, the V coefficients in H), W = V_{j+1} H_{j+1,j}; the deficiency test of
   ``oracle.gmres``.  So Op V_j = C B_j + V_{j+1} Hbar_j.
5. Least squares over span([U, V]): with R orthogonal to C the problem
   min || [0; S e_1] - [[D, B], [0, Hbar]] [y1; y2] || splits into the block
   GMRES problem y2 = argmin ||E_1 S - Hbar y2|| and y1 = -D^{-1} B y2; stop the
   cycle when every column's least-squares residual is <= tol ||b_c||.
   X <- X + P (V y2 - U (B y2)).
6. New recycled space (every cycle with steps, the harmonic Ritz vectors of
   Op on span(Vhat)): Vhat = [U D, V_1..V_j], What = [C, V_1..V_{j+1}],
   G = [[D, B], [0, Hbar]] with D = diag(1/||u_i||) (without C: Vhat = V_1..V_j,
   What = V_1..V_{j+1}, G = Hbar); the eigenpairs of
   G^T (What^T Vhat) z = mu G^T G z (mu = 1/theta, theta the harmonic Ritz
   values), the kr with the largest |mu| (see ``harmonic_select``); then
   Y = Vhat P_k, G P_k = Q R (thin QR), C <- What Q, U <- Y R^{-1}.
7. When the system is solved, U~ <- U for the next call.

With kr = 0 nothing is recycled and the steps are those of ``block_gmres``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .gmres import qr_positive, column_sines, DEP_SINE, STEP_DEF


@dataclasses.dataclass
class GcroInfo:
    converged: bool
    breakdown: bool
    steps: List[int]
    relres: np.ndarray
    recycled: List[int]  # recycled dimension after each cycle
    harmonic: List[np.ndarray]  # the selected mu values of each update


REAL_MU = 1e-10  # |Im mu| <= REAL_MU max|mu| counts as a real eigenvalue


def harmonic_select(G, WtV, kr):
    """The recycled directions P_k (N x kc, kc <= kr): eigenvectors z of
    G^T WtV z = mu G^T G z taken by decreasing |mu| (equal magnitudes by the
    library's order).  A real mu (|Im mu| <= REAL_MU max|mu|) gives Re z after
    z is scaled to unit norm with its largest entry real and positive; a complex
    pair gives Re z, Im z of its member with positive imaginary part; a pair
    that does not fit in what is left of kr ends the selection.  Returns (P_k,
    the selected mu)."""
    if kr <= 0:
        return np.zeros((G.shape[1], 0)), np.zeros(0)
    mu, Z = sla.eig(G.T @ WtV, G.T @ G)
    ok = np.isfinite(mu)
    if not np.any(ok):
        return np.zeros((G.shape[1], 0)), np.zeros(0)
    thr = REAL_MU * np.abs(mu[ok]).max()
    order = [i for i in np.argsort(-np.abs(np.where(ok, mu, 0.0)), kind="stable") if ok[i]]
    cols, picked, used = [], [], set()
    for i in order:
        if len(cols) >= kr:
            break
        if i in used:
            continue
        if abs(mu[i].imag) <= thr:
            z = Z[:, i] / np.linalg.norm(Z[:, i])
            t = int(np.argmax(np.abs(z)))
            z = z * (np.conj(z[t]) / abs(z[t]))
            cols.append(z.real)
            picked.append(mu[i])
            used.add(i)
            continue
        # the conjugate partner: the unused index with mu closest to conj(mu_i)
        rest = [t for t in order if t not in used and t != i]
        j = min(rest, key=lambda t: abs(mu[t] - np.conj(mu[i])))
        if len(cols) + 2 > kr:
            break
        z = Z[:, i] if mu[i].imag > 0 else Z[:, j]
        cols += [z.real, z.imag]
        picked += [mu[i], mu[j]]
        used |= {i, j}
    if not cols:
        return np.zeros((G.shape[1], 0)), np.zeros(0)
    return np.column_stack(cols), np.array(picked)


def block_gcrodr(A_apply, P_apply, B, m=30, kr=8, tol=1e-8, max_cycles=20, fixed_steps=None, recycle=None):
    """Solve A X = B by block GCRO-DR(m, kr), right-preconditioned by P.

    ``recycle``: a dict whose key "U" holds U~ (n x kc) from an earlier call (or
    None) and receives the recycled basis of this one.  ``fixed_steps`` forces
    the block steps of each cycle (replay of a solver under test).  B must have
    no zero column.  Returns (X, GcroInfo)."""
    if recycle is None:
        recycle = {}
    n, k = B.shape
    dt = np.result_type(B.dtype, np.float64)
    bnorm = np.linalg.norm(B, axis=0)
    if not np.all(bnorm > 0.0):
        raise ValueError("zero right-hand side column")
    info = GcroInfo(False, False, [], np.zeros(k), [], [])
    X = np.zeros((n, k), dtype=dt)
    C = U = None
    Ut = recycle.get("U")
    if Ut is not None and Ut.shape[1] > 0:
        Cm = A_apply(P_apply(Ut))
        Q, R = qr_positive(Cm)
        C = Q
        U = sla.solve_triangular(R, Ut.T, trans="T", lower=False).T  # Ut R^{-1}
    ncycles = max_cycles if fixed_steps is None else len(fixed_steps)
    for cycle in range(ncycles + 1):
        R = B - A_apply(X)
        if C is not None:
            T = C.conj().T @ R
            X = X + P_apply(U @ T)
            R = R - C @ T
        rel = np.linalg.norm(R, axis=0) / bnorm
        if not np.all(np.isfinite(rel)):
            break
        if fixed_steps is None and np.all(rel <= tol):
            info.converged = True
            break
        if cycle == ncycles:
            break
        V1, S = qr_positive(R)
        if not np.all(column_sines(R, S) > DEP_SINE):
            info.breakdown = True
            info.steps.append(0)
            break
        kc = 0 if C is None else C.shape[1]
        V = [V1]
        Hbar = np.zeros(((m + 1) * k, m * k), dtype=dt)
        Bc = np.zeros((kc, m * k), dtype=dt)
        Gr = np.zeros(((m + 1) * k, k), dtype=dt)
        Gr[:k, :] = S
        nsteps = m if fixed_steps is None else fixed_steps[cycle]
        Y = None
        j_done = 0
        deficient = False
        for j in range(nsteps):
            W = A_apply(P_apply(V[j]))
            wscale = np.linalg.norm(W, axis=0).max()
            basis = ([C] if C is not None else []) + V
            Vcat = np.hstack(basis)
            for _ in range(2):
                Hp = Vcat.conj().T @ W
                W = W - Vcat @ Hp
                Bc[:, j * k:(j + 1) * k] += Hp[:kc]
                Hbar[: (j + 1) * k, j * k:(j + 1) * k] += Hp[kc:]
            Vn, Hd = qr_positive(W)
            deficient = (np.abs(np.diag(Hd)).min() <= STEP_DEF * wscale
                         or not np.all(column_sines(W, Hd) > DEP_SINE))
            if deficient:
                Hd = np.zeros((k, k), dtype=dt)
                Vn = np.zeros((n, k), dtype=dt)
            Hbar[(j + 1) * k:(j + 2) * k, j * k:(j + 1) * k] = Hd
            V.append(Vn)
            Hj = Hbar[: (j + 2) * k, : (j + 1) * k]
            Y, *_ = np.linalg.lstsq(Hj, Gr[: (j + 2) * k, :], rcond=None)
            est = np.linalg.norm(Gr[: (j + 2) * k, :] - Hj @ Y, axis=0) / bnorm
            j_done = j + 1
            if deficient:
                break
            if fixed_steps is None and np.all(est <= tol):
                break
        info.steps.append(j_done)
        if j_done == 0:
            continue
        jk = j_done * k
        z = np.hstack(V[:j_done]) @ Y
        if C is not None:
            z = z - U @ (Bc[:, :jk] @ Y)
        X = X + P_apply(z)
        # the recycled space for the next cycle and the next system
        Hb = Hbar[: jk + k, : jk]
        if C is None:
            Vhat = np.hstack(V[:j_done])
            What = np.hstack(V[: j_done + 1])
            G = Hb
            WtV = np.vstack([np.eye(jk), np.zeros((k, jk))])
        else:
            d = 1.0 / np.linalg.norm(U, axis=0)
            Vhat = np.hstack([U * d[None, :]] + V[:j_done])
            What = np.hstack([C] + V[: j_done + 1])
            G = np.block([[np.diag(d), Bc[:, :jk]], [np.zeros((jk + k, kc)), Hb]])
            WtV = What.conj().T @ Vhat
        Pk, mu = harmonic_select(G, WtV, kr)
        info.harmonic.append(mu)
        if Pk.shape[1] > 0:
            Yk = Vhat @ Pk
            Q, Rk = qr_positive(G @ Pk)
            C = What @ Q
            U = sla.solve_triangular(Rk, Yk.T, trans="T", lower=False).T
        info.recycled.append(0 if C is None else C.shape[1])
    R = B - A_apply(X)
    info.relres = np.linalg.norm(R, axis=0) / bnorm
    if fixed_steps is None:
        info.converged = bool(np.all(info.relres <= tol))
    recycle["U"] = U
    return X, info
