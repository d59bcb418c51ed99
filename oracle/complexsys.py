"""Complex points — test infrastructure.

The expansion points of the paper's gyroscope example (Section 3) are complex:
with s = 2 pi f sqrt(-1), the coefficients s^2 and s^2 d are real and s theta,
s theta d are imaginary.  A = sum_t c_t T_t then has complex values on the
fixed union pattern of the real terms (plus the diagonal), and every step of
the method is taken in complex arithmetic here:

* SPAI (Section 2.2): column j solves min || e_j(I_j) - A(I_j, J_j) p ||_2 over
  complex p, by the library's least squares (``numpy.linalg.lstsq``);
* U-diag update (Section 2.3, first approach):
  q_i = argmin_q ||A(1) e_i - q A(l) e_i||_2 = (a_l^H a_1) / (a_l^H a_l), the
  closed form written out, and P_l = diag(q) P_1;
* block GMRES: ``oracle.gmres.block_gmres`` runs on complex blocks as it stands.

The real form (``real_form_csr``, ``real_form``, ``complex_of``) is the map
z -> [[Re z, -Im z], [Im z, Re z]] on entries and x_i -> (Re x_i, Im x_i) on
rows; it is used only to compare with a solver that works in real arithmetic.
"""
from __future__ import annotations

import numpy as np

from .assemble import union_pattern, affine_values


class ComplexAssembled:
    """A = sum_t c_t T_t (complex c_t) of a job with ``aterms`` on its union pattern."""

    def __init__(self, job):
        self.n = job.n
        self.terms = job.aterms
        self.rowptr, self.col, self.maps = union_pattern(job.n, self.terms)
        self.nnz = int(self.rowptr[-1])

    def values(self, coef):
        """Complex values of A at the coefficient vector ``coef`` (terms in list order)."""
        return affine_values(self.terms, self.maps, self.nnz, np.asarray(coef, dtype=np.complex128))


def to_dense(n, rowptr, col, val):
    A = np.zeros((n, n), dtype=np.result_type(val.dtype, np.float64))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            A[i, col[e]] += val[e]
    return A


def matvec(n, rowptr, col, val, X):
    """A X for a CSR matrix (plain row loops over numpy rows of X)."""
    X = np.asarray(X)
    Y = np.zeros((n,) + X.shape[1:], dtype=np.result_type(val.dtype, X.dtype))
    for i in range(n):
        sl = slice(rowptr[i], rowptr[i + 1])
        Y[i] = val[sl] @ X[col[sl]]
    return Y


def real_form_csr(n, rowptr, col, val):
    """The real form of an n x n complex CSR matrix: every stored entry z at
    (i, j) becomes the whole 2x2 block [[Re z, -Im z], [Im z, Re z]] at rows
    2i, 2i+1 and columns 2j, 2j+1 (zeros kept).  Returns (rowptr, col, val) of
    order 2n, columns sorted."""
    val = np.asarray(val, dtype=np.complex128)
    rp = np.zeros(2 * n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        sl = slice(rowptr[i], rowptr[i + 1])
        c = np.asarray(col[sl], dtype=np.int64)
        z = val[sl]
        r0c = np.empty(2 * c.size, dtype=np.int64)
        r0c[0::2] = 2 * c
        r0c[1::2] = 2 * c + 1
        r0v = np.empty(2 * c.size)
        r0v[0::2] = z.real
        r0v[1::2] = -z.imag
        r1v = np.empty(2 * c.size)
        r1v[0::2] = z.imag
        r1v[1::2] = z.real
        cols += [r0c, r0c]
        vals += [r0v, r1v]
        rp[2 * i + 1] = rp[2 * i] + 2 * c.size
        rp[2 * i + 2] = rp[2 * i + 1] + 2 * c.size
    return (rp.astype(np.int32), np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def real_form(X):
    """Rows of a complex vector or block as real rows: row 2i = Re, row 2i+1 = Im."""
    X = np.asarray(X, dtype=np.complex128)
    out = np.empty((2 * X.shape[0],) + X.shape[1:])
    out[0::2] = X.real
    out[1::2] = X.imag
    return out


def complex_of(Xr):
    """Inverse of ``real_form``."""
    Xr = np.asarray(Xr)
    return Xr[0::2] + 1j * Xr[1::2]


def spai_complex_column(n, rowptr, col, val, pat, j):
    """Column j of the complex SPAI on the index sets of ``pat`` (an
    ``oracle.spai.SpaiPattern`` of A's pattern).  Returns (p_j on J_j, rho_j)."""
    I, J = pat.I(j), pat.J(j)
    Ahat = np.zeros((I.size, J.size), dtype=np.complex128)
    jpos = {int(c): t for t, c in enumerate(J)}
    for a, i in enumerate(I):
        for e in range(rowptr[i], rowptr[i + 1]):
            t = jpos.get(int(col[e]))
            if t is not None:
                Ahat[a, t] = val[e]
    rhs = (I == j).astype(np.complex128)
    p, *_ = np.linalg.lstsq(Ahat, rhs, rcond=None)
    return p, float(np.linalg.norm(rhs - Ahat @ p))


def spai_complex(n, rowptr, col, val, pat, columns=None):
    """P = argmin ||I - A P||_F on ``pat`` in complex arithmetic: values in the
    pattern's CSR order (NaN outside ``columns``) and rho per column."""
    cols = range(n) if columns is None else columns
    pv = np.full(pat.J_row.size, np.nan + 0j)
    rho = np.full(n, np.nan)
    for j in cols:
        x, r = spai_complex_column(n, rowptr, col, val, pat, j)
        a, b = pat.J_colptr[j], pat.J_colptr[j + 1]
        pv[pat.P_slot[a:b]] = x
        rho[j] = r
    return pv, rho


def diag_factors_complex(n, rowptr, col, val_1, val_l):
    """q_i = (a_l^H a_1) / (a_l^H a_l) with a_1 = A(1) e_i, a_l = A(l) e_i (one
    pattern), and the residuals ||a_1 - q_i a_l||."""
    q = np.zeros(n, dtype=np.complex128)
    rho = np.zeros(n)
    cols = [[] for _ in range(n)]
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            cols[col[e]].append(e)
    for i in range(n):
        s = np.array(cols[i], dtype=np.int64)
        a_l = val_l[s]
        a_1 = val_1[s]
        num = 0j
        den = 0.0
        for t in range(s.size):
            num += np.conj(a_l[t]) * a_1[t]
            den += (np.conj(a_l[t]) * a_l[t]).real
        q[i] = num / den
        rho[i] = np.linalg.norm(a_1 - q[i] * a_l)
    return q, rho


def update_diag_complex(n, P_rowptr, P_val_1, q):
    """P_l = diag(q) P_1: row i of P_1 times q_i (same pattern)."""
    out = np.array(P_val_1, dtype=np.complex128, copy=True)
    for i in range(n):
        out[P_rowptr[i]:P_rowptr[i + 1]] *= q[i]
    return out
