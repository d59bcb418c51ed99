"""Cheap SPAI update — test infrastructure.

Paper, Section 2.3 (Table 1) and Section 2.4.  With P_1 a SPAI of the anchor
A(1), the first approach enforces A(1) P_1 ~= A(l) P_l with P_l = Q_l P_1 and
computes Q_l from the column-separable problem

    min_Q ||A(1) - A(l) Q||_F^2 = sum_i || A(1) e_i - A(l) q_i ||_2^2.

The paper leaves the sparsity pattern of Q open (it inherits an adaptive one
from its SPAI library).  Two fixed readings are implemented:

* ``diag``    q_i has the single entry i: q_i = <A(l) e_i, A(1) e_i> / ||A(l) e_i||^2,
              and P_l = diag(q) P_1 is P_1 with row i scaled by q_i;
* ``pattern`` q_i has the pattern J_i of the SPAI (same local problems as the
              SPAI with right-hand side A(1) e_i); P_l is applied as Q_l (P_1 X).

The second approach of Table 1 (right column: anchor A(l-1), Q_l from
min ||A(l-1) - A(l) Q||_F and P_l = Q_l P_{l-1}) is given for comparison, with
the ``diag`` reading of Q (``second_approach_diag``).
"""
from __future__ import annotations

import numpy as np

from .spai import solve_column, dense_block
from .sparse import transpose_pattern


def diag_factors(n, rowptr, col, val_1, val_l):
    """q_i = argmin_q ||A(1) e_i - q A(l) e_i||_2 for every i (both on one pattern).

    The one-unknown least-squares problem has the closed form
    q_i = <A(l) e_i, A(1) e_i> / <A(l) e_i, A(l) e_i>, written out here.
    """
    colptr, rowidx, slot = transpose_pattern(n, rowptr, col)
    q = np.zeros(n)
    for i in range(n):
        s = slot[colptr[i]:colptr[i + 1]]
        a_l = val_l[s]
        a_1 = val_1[s]
        num = 0.0
        den = 0.0
        for t in range(s.size):
            num += a_l[t] * a_1[t]
            den += a_l[t] * a_l[t]
        q[i] = num / den
    return q


def update_diag(n, P_rowptr, P_val_1, q):
    """P_l = diag(q) P_1: row i of P_1 scaled by q_i (same pattern)."""
    out = np.array(P_val_1, dtype=np.float64, copy=True)
    for i in range(n):
        out[P_rowptr[i]:P_rowptr[i + 1]] *= q[i]
    return out


def update_pattern(n, rowptr, col, val_1, val_l, pat, columns=None):
    """Q_l = argmin ||A(1) - A(l) Q||_F on the SPAI pattern; returns (Q values in pat's
    CSR order, rho per column)."""
    cols = range(n) if columns is None else columns
    qv = np.full(pat.J_row.size, np.nan)
    rho = np.full(n, np.nan)
    for i in cols:
        I = pat.I(i)
        a1 = dense_block(n, rowptr, col, val_1, I, np.array([i]))[:, 0]
        x, r = solve_column(n, rowptr, col, val_l, pat, i, rhs_full_column=lambda _I, a1=a1: a1)
        a, b = pat.J_colptr[i], pat.J_colptr[i + 1]
        qv[pat.P_slot[a:b]] = x
        rho[i] = r
    return qv, rho


def second_approach_diag(n, rowptr, col, vals, P_rowptr, P_val_1):
    """The second approach of Table 1 with a diagonal Q, over a sequence.

    vals[0], vals[1], ...: the values of A(1), A(2), ... on one pattern (A(1)
    is the matrix P_1 was built for).  For l >= 2 (vals index l - 1 >= 1):
    q_l = diag_factors(A(l-1), A(l)), i.e. the anchor is the previous matrix,
    and P_l = diag(q_l) P_{l-1}, taken literally as a row scaling of the
    previous preconditioner.  Returns the list [P_1, P_2, ...] of values in
    P's CSR order and the list [None, q_2, q_3, ...] of the step factors.
    """
    Ps = [np.array(P_val_1, dtype=np.float64, copy=True)]
    qs = [None]
    for l in range(1, len(vals)):
        q = diag_factors(n, rowptr, col, vals[l - 1], vals[l])
        Ps.append(update_diag(n, P_rowptr, Ps[-1], q))
        qs.append(q)
    return Ps, qs


def misfit_diag(n, rowptr, col, val_a, val_l):
    """Relative misfit of the U-diag update of A(l) against the anchor A(a):
    ||A(a) - A(l) diag(q)||_F / ||A(a)||_F with q = diag_factors(A(a), A(l)),
    summed column by column on the pattern."""
    q = diag_factors(n, rowptr, col, val_a, val_l)
    colptr, rowidx, slot = transpose_pattern(n, rowptr, col)
    num = 0.0
    for i in range(n):
        s = slot[colptr[i]:colptr[i + 1]]
        d = val_a[s] - q[i] * val_l[s]
        num += float(d @ d)
    return float(np.sqrt(num) / np.linalg.norm(val_a))


def plan_anchors(n, rowptr, col, vals, tol):
    """Re-anchoring of a sequence (first approach, U-diag): point 0 is the first
    anchor; the points are taken in order and a point whose misfit against the
    current anchor exceeds tol (or is not finite) becomes the next anchor (its
    preconditioner is rebuilt and later points are updated from it)."""
    anchors = [0]
    a = 0
    for l in range(1, len(vals)):
        r = misfit_diag(n, rowptr, col, vals[a], vals[l])
        if not (r <= tol):
            anchors.append(l)
            a = l
    return anchors


def update_adaptive(n, rowptr, col, val_1, val_l, pat, ep):
    """Adaptive pattern of Q (a reading of the paper's adaptive MSPAI pattern):
    every column first takes the diagonal factor q_i of ``diag_factors``; a
    column whose misfit ||A(1) e_i - q_i A(l) e_i|| exceeds ep ||A(1) e_i|| is
    escalated to the SPAI pattern J_i and solved as in ``update_pattern``.
    Returns (Q values in pat's CSR order, rho per column, escalated columns)."""
    q = diag_factors(n, rowptr, col, val_1, val_l)
    colptr, rowidx, slot = transpose_pattern(n, rowptr, col)
    qv = np.zeros(pat.J_row.size)
    rho = np.zeros(n)
    esc = []
    for i in range(n):
        s = slot[colptr[i]:colptr[i + 1]]
        a1 = val_1[s]
        d = a1 - q[i] * val_l[s]
        r = float(np.sqrt(d @ d))
        if not (r <= ep * float(np.sqrt(a1 @ a1))):
            esc.append(i)
            continue
        a, b = pat.J_colptr[i], pat.J_colptr[i + 1]
        qv[pat.P_slot[a:b][pat.J_row[a:b] == i]] = q[i]
        rho[i] = r
    if esc:
        qe, re = update_pattern(n, rowptr, col, val_1, val_l, pat, columns=esc)
        for i in esc:
            a, b = pat.J_colptr[i], pat.J_colptr[i + 1]
            qv[pat.P_slot[a:b]] = qe[pat.P_slot[a:b]]
            rho[i] = re[i]
    return qv, rho, esc
