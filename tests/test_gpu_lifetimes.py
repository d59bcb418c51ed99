"""Handles may be destroyed in any order: a context outlives its problems and
servers, a problem its preconditioners (reference counts in the library)."""
import ctypes as C

import pytest
import torch

from synth import config0
from tests._helpers import ctx as make_ctx

pytestmark = pytest.mark.gpu


def _problem_and_spai(ctx):
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    h = pb.spai_build(job.s, job.p_list[0])
    return job, pb, h


@pytest.mark.parametrize("order", ["problem_first", "context_first", "natural"])
def test_destroy_in_any_order(gpu_lib, order):
    from paper_1809_06574_amd import lib as L
    ctx = make_ctx()
    job, pb, h = _problem_and_spai(ctx)
    B = torch.as_tensor(job.B, device="cuda")
    X, st, rc = pb.block_solve(h, job.s, job.p_list[0], B)
    assert rc == 0
    if order == "problem_first":
        pb.close()
        h.update(job.s, job.p_list[1])  # the preconditioner still works on its problem's data
        h.close()
        ctx.close()
    elif order == "context_first":
        ctx.close()
        h.close()
        pb.close()
    else:
        h.close()
        pb.close()
        ctx.close()
    # a fresh context afterwards works
    ctx2 = make_ctx()
    job, pb2, h2 = _problem_and_spai(ctx2)
    X2, st2, rc2 = pb2.block_solve(h2, job.s, job.p_list[0], torch.as_tensor(job.B, device="cuda"))
    assert rc2 == 0 and torch.equal(X, X2)


def test_stream_replaced_and_destroyed(gpu_lib):
    """A context's stream replaced (pmor_ctx_set_stream) and the old one destroyed
    (hipStreamDestroy): device blocks the library released on the old stream are
    handed out again afterwards without touching it, and the results equal those
    of a context that kept one stream."""
    from paper_1809_06574_amd import lib as L, Problem
    hip = C.CDLL("libamdhip64.so")
    ctx = make_ctx()
    job = config0()
    B = torch.as_tensor(job.B, device="cuda")
    ref_pb = Problem(ctx, job.terms)
    ref_h = ref_pb.spai_build(job.s, job.p_list[1])
    Xr, _, _ = ref_pb.block_solve(ref_h, job.s, job.p_list[1], B)
    torch.cuda.synchronize()
    side = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(side)) == 0
    assert L.pmor_ctx_set_stream(ctx.handle, side) == 0
    for _ in range(3):  # blocks released on the side stream
        pb = Problem(ctx, job.terms)
        h = pb.spai_build(job.s, job.p_list[0])
        pb.block_solve(h, job.s, job.p_list[0], B)
        h.close()
        pb.close()
    assert L.pmor_ctx_set_stream(ctx.handle, C.c_void_p(ctx.stream.cuda_stream)) == 0
    assert hip.hipStreamDestroy(side) == 0
    pb = Problem(ctx, job.terms)
    h = pb.spai_build(job.s, job.p_list[1])
    X, st, rc = pb.block_solve(h, job.s, job.p_list[1], B)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(X, Xr)
