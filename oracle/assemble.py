"""Assembly of A(s,p) = s^2 M(p) + s D(p) + K(p) — test infrastructure.

The frequency-domain matrix of the second-order system (paper, Section 1.1
and eq. loewner_eq2 in Section 1.2), with each coefficient matrix affine in
the parameter: M(p) = M0 + p M1, D(p) = D0 + p D1, K(p) = K0 + p K1.
The general affine form of Section 1.1 (eq. affine_system),
A = A_0 + s~_1 A_1 + ... + s~_{w+1} A_{w+1}, is ``affine_values``: a list of
term matrices and one coefficient per term (the coefficient of A_0 is 1).

The pattern of A is the union of the term patterns plus the full diagonal.
Entries that cancel numerically stay in the pattern, so the pattern does not
depend on (s, p) and is the same for every matrix of a sequence.
"""
from __future__ import annotations

import numpy as np

ROLES = ("M0", "M1", "D0", "D1", "K0", "K1")


def union_pattern(n, terms):
    """CSR pattern of the union of ``terms`` (dict role -> CSR, or a list of CSR
    indexed by position) and the diagonal.

    Returns (rowptr, col, maps) where maps[key][e] is the position of A-slot e in
    that term's value array, or -1 where the term has no entry.
    """
    keys = [np.arange(n, dtype=np.int64) * (n + 1)]  # diagonal keys i*n + i
    term_keys = {}
    names = [r for r in ROLES if r in terms] if isinstance(terms, dict) else list(range(len(terms)))
    for role in names:
        T = terms[role]
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(T.rowptr.astype(np.int64)))
        tk = rows * n + T.col.astype(np.int64)
        term_keys[role] = tk
        keys.append(tk)
    allk = np.unique(np.concatenate(keys))  # sorted: by row, then column
    rows = allk // n
    col = (allk % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    maps = {}
    for role, tk in term_keys.items():
        pos = np.searchsorted(tk, allk)  # term keys are sorted (CSR with sorted columns)
        pos_c = np.minimum(pos, tk.size - 1)
        hit = (pos < tk.size) & (tk[pos_c] == allk)
        maps[role] = np.where(hit, pos_c, -1).astype(np.int32)
    return rowptr.astype(np.int32), col, maps


def term_values_on_pattern(terms, maps, nnz):
    """Each term's values scattered onto the union pattern (0 where absent)."""
    out = {}
    for role in ROLES:
        if role in maps:
            m = maps[role]
            v = np.zeros(nnz)
            v[m >= 0] = terms[role].val[m[m >= 0]]
            out[role] = v
        else:
            out[role] = np.zeros(nnz)
    return out


def affine_values(terms, maps, nnz, coef):
    """Values of sum_t coef[t] T_t on the union pattern (terms: list of CSR, maps by
    list position), the terms added in list order."""
    out = np.zeros(nnz)
    for t, T in enumerate(terms):
        m = maps[t]
        v = np.zeros(nnz)
        v[m >= 0] = T.val[m[m >= 0]]
        out = out + coef[t] * v
    return out


def assemble_values(terms, maps, nnz, s, p):
    """Values of A(s,p) on the union pattern: s^2 (M0 + p M1) + s (D0 + p D1) + (K0 + p K1)."""
    t = term_values_on_pattern(terms, maps, nnz)
    Mv = t["M0"] + p * t["M1"]
    Dv = t["D0"] + p * t["D1"]
    Kv = t["K0"] + p * t["K1"]
    return (s * s) * Mv + s * Dv + Kv


class Assembled:
    """A of one job on its fixed union pattern: at (s, p) for a job of roles, at a
    coefficient vector for an affine job (``job.aterms``)."""

    def __init__(self, job):
        self.n = job.n
        self.affine = getattr(job, "aterms", None) is not None
        self.terms = job.aterms if self.affine else job.terms
        self.rowptr, self.col, self.maps = union_pattern(job.n, self.terms)
        self.nnz = int(self.rowptr[-1])

    def values(self, s, p):
        assert not self.affine, "an affine job takes coefficient vectors (values_c)"
        return assemble_values(self.terms, self.maps, self.nnz, s, p)

    def values_c(self, coef):
        assert self.affine, "values_c is for affine jobs"
        return affine_values(self.terms, self.maps, self.nnz, coef)
