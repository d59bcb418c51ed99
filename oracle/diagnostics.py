"""Diagnostic norms — test infrastructure.

Paper, Section 3.1 and Table 2: the update pays off when ||I - A(l)||_F is
large while ||A(1) - A(l)||_F is small.  ||I - A P||_F^2 is the SPAI objective
of Section 2.2 and equals the sum of the squared column residuals.
"""
from __future__ import annotations

import numpy as np


def fro_I_minus_A(n, rowptr, col, val):
    """||I - A||_F for A in CSR."""
    tot = 0.0
    for i in range(n):
        has_diag = False
        for e in range(rowptr[i], rowptr[i + 1]):
            x = val[e]
            if col[e] == i:
                has_diag = True
                x = 1.0 - x
            tot += x * x
        if not has_diag:
            tot += 1.0
    return float(np.sqrt(tot))


def fro_diff(val_1, val_l):
    """||A(1) - A(l)||_F for two matrices on the same pattern."""
    d = np.asarray(val_1) - np.asarray(val_l)
    return float(np.sqrt(np.sum(d * d)))


def fro_from_residuals(rho):
    """||I - A P||_F (or ||A(1) - A(l) Q||_F) from the column residuals."""
    rho = np.asarray(rho)
    return float(np.sqrt(np.sum(rho * rho)))
