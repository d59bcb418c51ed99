"""pmor_table2_norms_noalloc (the entry point for callers that cannot allocate)
against pmor_table2_norms, through the C ABI: two calls in a row, the second on
a smaller problem, each within 1e-14 relative of the allocating call (both sum
the same entry values in the same row split); the dense Frobenius norms of the
oracle's assembled matrices agree within 1e-12; repeated calls leave the
device's free memory unchanged."""
import ctypes as C

import numpy as np
import pytest
import torch

from synth import config0, tiny_random_job
from oracle.assemble import Assembled
from oracle.sparse import to_dense
from tests._helpers import ctx as make_ctx

pytestmark = pytest.mark.gpu


def _norms(lib, pb, fn, s1, p1, s2, p2):
    a, b = C.c_double(), C.c_double()
    rc = getattr(lib, fn)(pb.handle, s1, p1, s2, p2, C.byref(a), C.byref(b))
    assert rc == 0, (fn, rc, lib.pmor_last_error())
    return a.value, b.value


def _dense(job, s, p):
    asm = Assembled(job)
    return to_dense(job.n, asm.rowptr, asm.col, asm.values(s, p))


def test_noalloc_matches_the_allocating_call(gpu_lib):
    from paper_1809_06574_amd import Problem
    L = gpu_lib
    ctx = make_ctx()
    jobs = [config0(), tiny_random_job(64, 0.06, 2, k=3, roles=("M0", "M1", "D0", "D1", "K0", "K1"))]
    assert jobs[1].n < jobs[0].n
    for job in jobs:  # two calls in a row, the second with a smaller input
        pb = Problem(ctx, job.terms)
        s, p1, p2 = job.s, float(job.p_list[0]), float(job.p_list[-1])
        print(f"no-alloc norms: {job.name} n={job.n} nnz={pb.nnz}", flush=True)
        got = _norms(L, pb, "pmor_table2_norms_noalloc", s, p1, s, p2)
        want = _norms(L, pb, "pmor_table2_norms", s, p1, s, p2)
        for g, w in zip(got, want):
            assert abs(g - w) <= 1e-14 * max(abs(w), 1e-300), (got, want)
        A1, A2 = _dense(job, s, p1), _dense(job, s, p2)
        assert got[0] == pytest.approx(np.linalg.norm(np.eye(job.n) - A2), rel=1e-12)
        assert got[1] == pytest.approx(np.linalg.norm(A1 - A2), rel=1e-12)
        # the same point twice: ||A1 - A1|| = 0 exactly
        assert _norms(L, pb, "pmor_table2_norms_noalloc", s, p1, s, p1)[1] == 0.0
        pb.close()


def test_noalloc_allocates_nothing(gpu_lib):
    from paper_1809_06574_amd import Problem
    ctx = make_ctx()
    job = config0()
    pb = Problem(ctx, job.terms)
    pb.table2_norms_noalloc(job.s, 0.1, job.s, 0.4)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    vals = [pb.table2_norms_noalloc(job.s, 0.1, job.s, 0.1 + 0.1 * r) for r in range(5)]
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert vals[0][1] == 0.0 and all(v[1] > 0.0 for v in vals[1:])
    pb.close()
