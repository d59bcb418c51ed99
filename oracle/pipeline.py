"""One job's sequence of parametric solves — test infrastructure.

Paper, Section 2.3 (eq. general_sq) and Section 3: for the points
(s, p_1), ..., (s, p_z) of a job, assemble A(l), get a preconditioner
(SPAI of A(1) at l = 1; then either a rebuild or the first-approach update
P_l = Q_l P_1 anchored at A(1)), and solve A(l) X(l) = B with block GMRES.
"""
from __future__ import annotations

import time

import numpy as np

from .assemble import Assembled
from .spai import SpaiPattern, spai_build
from .update import diag_factors, update_diag, update_pattern
from .sparse import to_scipy
from .gmres import block_gmres


class JobOracle:
    def __init__(self, job):
        self.job = job
        self.asm = Assembled(job)
        self.pat = SpaiPattern(job.n, self.asm.rowptr, self.asm.col, explicit=job.pattern)

    def A(self, p):
        v = self.asm.values(self.job.s, p)
        return v, to_scipy(self.job.n, self.asm.rowptr, self.asm.col, v)

    def A_at(self, l):
        """A at point l of the job: (s, p_l), or the coefficient vector coefs[l] of an
        affine job."""
        if self.asm.affine:
            v = self.asm.values_c(self.job.coefs[l])
            return v, to_scipy(self.job.n, self.asm.rowptr, self.asm.col, v)
        return self.A(self.job.p_list[l])

    def spai(self, val):
        return spai_build(self.job.n, self.asm.rowptr, self.asm.col, val, self.pat)

    def P(self, pv):
        return to_scipy(self.job.n, self.pat.P_rowptr, self.pat.P_col, pv)

    def run(self, policy="update", update_kind="diag", m=30, tol=1e-8, max_cycles=20,
            points=None):
        """Solve every point; returns a list of dicts (X, info, timings)."""
        job = self.job
        pts = range(len(job.p_list)) if points is None else points
        out = []
        val1 = None
        pv1 = None
        for l in pts:
            t0 = time.perf_counter()
            val, A = self.A_at(l)
            t1 = time.perf_counter()
            if pv1 is None or policy == "rebuild":
                pv, _ = self.spai(val)
                if pv1 is None:
                    val1, pv1 = val, pv
                Papply = self.P(pv).__matmul__
            elif update_kind == "diag":
                q = diag_factors(job.n, self.asm.rowptr, self.asm.col, val1, val)
                Papply = self.P(update_diag(job.n, self.pat.P_rowptr, pv1, q)).__matmul__
            else:
                qv, _ = update_pattern(job.n, self.asm.rowptr, self.asm.col, val1, val, self.pat)
                Q = self.P(qv)
                P1 = self.P(pv1)
                Papply = (lambda Xb, Q=Q, P1=P1: Q @ (P1 @ Xb))
            t2 = time.perf_counter()
            X, info = block_gmres(A.__matmul__, Papply, job.B, m=m, tol=tol, max_cycles=max_cycles)
            t3 = time.perf_counter()
            out.append({"X": X, "info": info, "t_assemble": t1 - t0, "t_precond": t2 - t1,
                        "t_solve": t3 - t2})
        return out
