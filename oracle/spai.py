"""Sparse approximate inverse (SPAI) by Frobenius minimisation — test infrastructure.

Paper, Section 2.2: min_P ||I - A P||_F^2 = sum_j ||e_j - A p_j||_2^2, so every
column p_j of P is an independent least-squares problem.  With the allowed
nonzero rows J_j of p_j, only the rows I_j of A(:, J_j) that hold a nonzero
(the "shadow" of J_j) enter the problem, so column j solves the small dense
problem  min || e_j(I_j) - A(I_j, J_j) p ||_2  and its residual rho_j is also
the residual of the full column problem (rows outside I_j contribute e_j's
entries only, and j is in I_j whenever A(j, c) != 0 for some c in J_j).

The least-squares problems are solved by Householder QR (reflectors in the
LAPACK larfg convention), then back substitution with R.  A column whose R has
a pivot |R_kk| <= 10 |I_j| eps max|R| is reported as singular.
"""
from __future__ import annotations

import numpy as np

from .sparse import transpose_pattern, csc_to_csr

EPS = np.finfo(np.float64).eps


class SingularColumn(Exception):
    def __init__(self, column):
        super().__init__(f"rank-deficient local least-squares problem in column {column}")
        self.column = column


def pattern_of_A(n, rowptr, col):
    """J_j = rows holding a structural nonzero in column j of A, plus j (CSC, sorted)."""
    colptr, rowidx, _ = transpose_pattern(n, rowptr, col)
    cp = [0]
    rows = []
    for j in range(n):
        r = rowidx[colptr[j]:colptr[j + 1]]
        if not np.any(r == j):
            r = np.sort(np.append(r, j))
        rows.append(r)
        cp.append(cp[-1] + r.size)
    return np.array(cp, dtype=np.int32), np.concatenate(rows).astype(np.int32)


def shadow(n, J_colptr, J_row, rowptr, col):
    """I_j = sorted union over c in J_j of the rows of A(:, c) (CSC, sorted)."""
    colptr, rowidx, _ = transpose_pattern(n, rowptr, col)
    cp = [0]
    rows = []
    for j in range(n):
        Jj = J_row[J_colptr[j]:J_colptr[j + 1]]
        parts = [rowidx[colptr[c]:colptr[c + 1]] for c in Jj]
        r = np.unique(np.concatenate(parts)) if parts else np.zeros(0, dtype=np.int32)
        rows.append(r.astype(np.int32))
        cp.append(cp[-1] + r.size)
    return np.array(cp, dtype=np.int64), np.concatenate(rows).astype(np.int32)


def dense_block(n, rowptr, col, val, I, J):
    """A(I, J) as a dense |I| x |J| array (plain loops)."""
    out = np.zeros((len(I), len(J)))
    jpos = {int(c): t for t, c in enumerate(J)}
    for a, i in enumerate(I):
        for e in range(rowptr[i], rowptr[i + 1]):
            t = jpos.get(int(col[e]))
            if t is not None:
                out[a, t] = val[e]
    return out


def householder(x):
    """Reflector H = I - tau v v^T with v[0] = 1 such that H x = beta e_1.

    LAPACK larfg convention: beta = -sign(x0) ||x|| (sign(0) = +1); if x[1:] == 0
    then tau = 0 and H = I.
    """
    alpha = float(x[0])
    sigma = float(np.dot(x[1:], x[1:]))
    v = np.zeros(x.size); v[0] = 1.0
    if sigma == 0.0:
        return v, 0.0, alpha
    norm = np.sqrt(alpha * alpha + sigma)
    beta = -norm if alpha >= 0.0 else norm
    v[1:] = x[1:] / (alpha - beta)
    tau = (beta - alpha) / beta
    return v, tau, beta


def back_substitute(R, y):
    nj = R.shape[0]
    p = np.zeros(nj)
    for i in range(nj - 1, -1, -1):
        p[i] = (y[i] - np.dot(R[i, i + 1:], p[i + 1:])) / R[i, i]
    return p


def householder_lstsq(Ahat, rhs, column=-1):
    """min ||rhs - Ahat p||_2 by Householder QR; returns (p, rho = residual norm)."""
    R = np.array(Ahat, dtype=np.float64, copy=True)
    y = np.array(rhs, dtype=np.float64, copy=True)
    m, nj = R.shape
    if m < nj:
        raise SingularColumn(column)
    for k in range(nj):
        v, tau, beta = householder(R[k:, k])
        if tau != 0.0:
            R[k:, k:] -= tau * np.outer(v, v @ R[k:, k:])
            y[k:] -= tau * v * (v @ y[k:])
        R[k, k] = beta
        R[k + 1:, k] = 0.0
    Rt = np.triu(R[:nj, :nj])
    d = np.abs(np.diag(Rt))
    if nj and (d.min() <= 10.0 * m * EPS * np.abs(Rt).max() or not np.all(np.isfinite(Rt))):
        raise SingularColumn(column)
    return back_substitute(Rt, y[:nj]), float(np.linalg.norm(y[nj:]))


class SpaiPattern:
    """The per-column index sets of one job (fixed for the whole sequence)."""

    def __init__(self, n, rowptr, col, explicit=None):
        self.n = n
        if explicit is None:
            self.J_colptr, self.J_row = pattern_of_A(n, rowptr, col)
        else:
            self.J_colptr = np.asarray(explicit[0], dtype=np.int32)
            self.J_row = np.asarray(explicit[1], dtype=np.int32)
        self.I_colptr, self.I_row = shadow(n, self.J_colptr, self.J_row, rowptr, col)
        # P is stored in CSR; slot maps column-computed entries into it
        self.P_rowptr, self.P_col, self.P_slot = csc_to_csr(n, self.J_colptr, self.J_row)

    def J(self, j):
        return self.J_row[self.J_colptr[j]:self.J_colptr[j + 1]]

    def I(self, j):
        return self.I_row[self.I_colptr[j]:self.I_colptr[j + 1]]


def solve_column(n, rowptr, col, val, pat, j, rhs_full_column=None):
    """Column j of min ||R - A X||_F on pattern J_j.

    ``rhs_full_column`` is a function i -> R(i, j) on the shadow rows; None means
    the identity (SPAI: e_j).  Returns (x_j on J_j, rho_j).
    """
    I = pat.I(j); J = pat.J(j)
    Ahat = dense_block(n, rowptr, col, val, I, J)
    if rhs_full_column is None:
        rhs = (I == j).astype(np.float64)
    else:
        rhs = rhs_full_column(I)
    return householder_lstsq(Ahat, rhs, column=j)


def spai_build(n, rowptr, col, val, pat, columns=None):
    """P = argmin ||I - A P||_F on pattern ``pat``.

    Returns (P values in pat's CSR order, rho per column).  ``columns`` restricts
    the work to a subset (the other entries stay NaN) for sampled checks.
    """
    cols = range(n) if columns is None else columns
    pv = np.full(pat.J_row.size, np.nan)
    rho = np.full(n, np.nan)
    for j in cols:
        x, r = solve_column(n, rowptr, col, val, pat, j)
        a, b = pat.J_colptr[j], pat.J_colptr[j + 1]
        pv[pat.P_slot[a:b]] = x
        rho[j] = r
    return pv, rho
