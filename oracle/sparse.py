"""Plain CSR helpers for the oracle (test infrastructure; no GPU code)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def check_csr(n, rowptr, col):
    """Raise ValueError unless (rowptr, col) is a valid 0-based CSR with sorted unique columns."""
    rowptr = np.asarray(rowptr); col = np.asarray(col)
    if rowptr.shape != (n + 1,) or rowptr[0] != 0:
        raise ValueError("bad rowptr")
    if np.any(np.diff(rowptr) < 0) or rowptr[-1] != col.size:
        raise ValueError("rowptr not monotone / nnz mismatch")
    if col.size and (col.min() < 0 or col.max() >= n):
        raise ValueError("column index out of range")
    for i in range(n):
        c = col[rowptr[i]:rowptr[i + 1]]
        if c.size > 1 and np.any(np.diff(c) <= 0):
            raise ValueError(f"row {i}: columns not strictly increasing")


def to_scipy(n, rowptr, col, val):
    return sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(rowptr)),
                         shape=(n, n))


def to_dense(n, rowptr, col, val):
    D = np.zeros((n, n))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            D[i, col[e]] = val[e]
    return D


def transpose_pattern(n, rowptr, col):
    """CSC view of a CSR pattern.

    Returns (colptr, rowidx, slot): column j holds rows rowidx[colptr[j]:colptr[j+1]]
    in ascending order, and slot[q] is the CSR position of CSC entry q.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64); col = np.asarray(col, dtype=np.int64)
    nnz = col.size
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    # stable sort by column keeps rows ascending inside each column
    order = np.argsort(col, kind="stable")
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(col, minlength=n), out=colptr[1:])
    assert colptr[-1] == nnz
    return colptr.astype(np.int32), rows[order].astype(np.int32), order.astype(np.int32)


def csc_to_csr(n, colptr, rowidx):
    """Transpose an explicit CSC pattern into CSR; also return the CSC->CSR slot map."""
    colptr = np.asarray(colptr, dtype=np.int64); rowidx = np.asarray(rowidx, dtype=np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    order = np.argsort(rowidx, kind="stable")  # by row, columns ascending within a row
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rowidx, minlength=n), out=rowptr[1:])
    csr_col = cols[order]
    slot = np.empty(rowidx.size, dtype=np.int64)
    slot[order] = np.arange(rowidx.size)
    return rowptr.astype(np.int32), csr_col.astype(np.int32), slot.astype(np.int32)
