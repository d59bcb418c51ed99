"""Block GMRES(m) with right preconditioning — test infrastructure.

Paper, Section 2.1: for A X = B with several right-hand sides available
together, a block Krylov method searches X - X0 in the block Krylov space
span{R0, A R0, A^2 R0, ...} of the block residual R0 = B - A X0.  With right
preconditioning (footnote of Section 2.2) the iteration runs on A P and the
solution is recovered as X = P X~.  The paper's own solver is block GCRO;
block GMRES(m) (the block Arnoldi process with a least-squares problem on the
block Hessenberg matrix, restarted every m block steps) is the solver built
here.  Steps, in order:

1. R = B - A X; stop if every column has ||r_c|| <= tol ||b_c||.
2. Thin QR  R = V_1 S  (positive diagonal of S, which makes it unique).
3. For j = 1..m:  Z = P V_j;  W = A Z;  two passes of classical Gram-Schmidt
   against [V_1..V_j] (H_{1:j, j} accumulates both passes' coefficients);
   thin QR  W = V_{j+1} H_{j+1, j};  Y_j = argmin ||E_1 S - Hbar_j Y||_F;
   stop the cycle when every column's least-squares residual is <= tol ||b_c||.
4. X = X + P [V_1..V_j] Y_j and go to 1 (a restart) unless converged.

Zero columns of B have the solution 0 and are left out of the block.

Complex systems (the expansion points of Section 3 are complex) take the same
steps in complex arithmetic: the Gram-Schmidt coefficients are V^H W, and the
QR factors carry a real positive diagonal (each column's unit-modulus phase
moved from R into Q).  For real data every step is the real one.

Dependent columns (the paper is silent; Section 2.1 only assumes the block
Krylov space has full dimension).  For a block Y with thin QR Y = Q S, the
ratio |S_cc| / ||y_c|| is the sine of the angle between column c and the span
of the columns before it.
* Cycle start: when a column of the residual block has a sine <= DEP_SINE
  (1e-6), the block is dependent (an exact or near duplicate right-hand side
  column, say).  Restarting cannot change that, so the solve stops with a
  breakdown and X keeps its current value, unless every column has already
  converged.  DEP_SINE sits well above the sine that Cholesky QR in FP64 can
  still resolve (about 1e-7 for blocks of up to 2^22 rows), so a solver using
  the Gram matrix and one using Householder reach the same verdict.
* Block step: the new block W (after Gram-Schmidt) is deficient when a column
  has a sine <= DEP_SINE, or |S_cc| <= 1e-14 max_c ||W_c|| with the norms
  taken before Gram-Schmidt (the block Krylov space stopped growing in that
  direction, e.g. a right-hand side inside an invariant subspace of A P).  The
  cycle takes H_{j+1,j} = 0 and ends there; its least-squares solution
  updates X as usual, and an unconverged solve restarts from the new residual.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

DEP_SINE = 1e-6  # sine below which a block column counts as dependent on the ones before it
STEP_DEF = 1e-14  # pivot of a new block, relative to max ||W_c|| before Gram-Schmidt


@dataclasses.dataclass
class GmresInfo:
    converged: bool
    breakdown: bool
    steps: List[int]  # block steps per cycle
    ls_history: List[np.ndarray]  # per block step: LS residual / ||b|| per column
    relres: np.ndarray  # final true relative residual per column
    hessenbergs: List[np.ndarray]


def qr_positive(W):
    """Thin QR with a real nonnegative diagonal in R (library Householder QR, then
    each column's phase, a sign for real data, moved from R into Q)."""
    Q, R = np.linalg.qr(W, mode="reduced")
    r = np.diag(R)
    mag = np.abs(r)
    d = np.where(mag > 0.0, r / np.where(mag > 0.0, mag, 1.0), 1.0)
    return Q * d[None, :], R * np.conj(d)[:, None]


def column_sines(Y, R):
    """|R_cc| / ||y_c|| for the thin QR Y = Q R: the sine of the angle between
    column c and the span of columns 0..c-1 (NaN for a zero column)."""
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.abs(np.diag(R)) / np.linalg.norm(Y, axis=0)


def block_gmres(A_apply: Callable, P_apply: Callable, B: np.ndarray, m: int = 30,
                tol: float = 1e-8, max_cycles: int = 20,
                fixed_steps: Optional[List[int]] = None):
    """Solve A X = B with block GMRES(m) right-preconditioned by P.

    ``fixed_steps`` forces the number of block steps of each cycle (the parity
    protocol: run exactly as many steps as the solver under test reported).
    Returns (X, GmresInfo).
    """
    n, k_all = B.shape
    dt = np.result_type(B.dtype, np.float64)
    X_all = np.zeros((n, k_all), dtype=dt)
    bnorm_all = np.linalg.norm(B, axis=0)
    active = np.nonzero(bnorm_all > 0.0)[0]
    info = GmresInfo(False, False, [], [], np.zeros(k_all), [])
    if active.size == 0:
        info.converged = True
        return X_all, info
    Bc = B[:, active]
    bnorm = bnorm_all[active]
    k = active.size
    X = np.zeros((n, k), dtype=dt)
    ncycles = max_cycles if fixed_steps is None else len(fixed_steps)
    for cycle in range(ncycles + 1):
        R = Bc - A_apply(X)
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
        V = [V1]
        Hbar = np.zeros(((m + 1) * k, m * k), dtype=dt)
        G = np.zeros(((m + 1) * k, k), dtype=dt)
        G[:k, :] = S
        nsteps = m if fixed_steps is None else fixed_steps[cycle]
        Y = None
        j_done = 0
        for j in range(nsteps):
            Z = P_apply(V[j])
            W = A_apply(Z)
            wscale = np.linalg.norm(W, axis=0).max()
            Vcat = np.hstack(V)
            for _ in range(2):
                Hp = Vcat.conj().T @ W
                W = W - Vcat @ Hp
                Hbar[: (j + 1) * k, j * k:(j + 1) * k] += Hp
            Vn, Hd = qr_positive(W)
            deficient = (np.abs(np.diag(Hd)).min() <= STEP_DEF * wscale
                         or not np.all(column_sines(W, Hd) > DEP_SINE))
            if deficient:
                Hd = np.zeros((k, k), dtype=dt)
                Vn = np.zeros((n, k), dtype=dt)
            Hbar[(j + 1) * k:(j + 2) * k, j * k:(j + 1) * k] = Hd
            V.append(Vn)
            Hj = Hbar[: (j + 2) * k, : (j + 1) * k]
            Gj = G[: (j + 2) * k, :]
            Y, *_ = np.linalg.lstsq(Hj, Gj, rcond=None)
            est = np.linalg.norm(Gj - Hj @ Y, axis=0) / bnorm
            info.ls_history.append(est)
            j_done = j + 1
            done = np.all(est <= tol)
            if deficient:
                break
            if fixed_steps is None and done:
                break
        info.steps.append(j_done)
        info.hessenbergs.append(Hbar[: (j_done + 1) * k, : j_done * k].copy())
        X = X + P_apply(np.hstack(V[:j_done]) @ Y)
    R = Bc - A_apply(X)
    rel = np.linalg.norm(R, axis=0) / bnorm
    info.relres[active] = rel
    info.converged = bool(np.all(rel <= tol)) if fixed_steps is None else info.converged
    X_all[:, active] = X
    return X_all, info
