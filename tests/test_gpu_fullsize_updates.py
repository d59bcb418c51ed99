"""The update options at the full grid size (64^3, n = 262144, k = 4, 20 points),
solved as the benchmark's comparison runs solve them (pmor_sequence_solve,
update policy, all points together): the second approach of Table 1 and the
adaptive Q pattern.

Bars: every column of every point at true relative residual <= 1e-8; the
second approach's running row scale and P_l after three chained updates
within 1e-12 relative of the oracle's literal chain diag(q_l) P_{l-1} (the
library keeps diag(q_l ... q_2) P_1: the same factors in another rounding
order); the adaptive run's per-point stats in the same form as the U-diag run.
"""
import numpy as np
import pytest
import torch

from synth import config1
from oracle.assemble import Assembled
from oracle.spai import SpaiPattern
from oracle.update import second_approach_diag
from oracle.sparse import to_scipy
from tests._helpers import np_, col_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1(gpu_lib):
    from paper_1809_06574_amd import Context, Problem
    job = config1()
    asm = Assembled(job)
    ctx = Context(0)
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    yield job, asm, pb, B
    pb.close()
    ctx.close()


def _check_residuals(job, asm, X):
    bn = np.linalg.norm(job.B, axis=0)
    for l, p in enumerate(job.p_list):
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
        rel = np.linalg.norm(job.B - A @ X[l], axis=0) / bn
        assert np.all(rel <= 1e-8 * 1.0001), (l, rel)


def test_c1_second_approach_true_residual_every_point(c1):
    job, asm, pb, B = c1
    X, stats = pb.sequence_solve(B, [job.s] * len(job.p_list), job.p_list, policy="update", approach="second")
    torch.cuda.synchronize()
    _check_residuals(job, asm, np_(X))
    assert all(st["cycles"] >= 1 and st["anchor"] == 0 for st in stats)


def test_c1_second_approach_chain_matches_the_oracle(c1):
    job, asm, pb, B = c1
    n = job.n
    pat = SpaiPattern(n, asm.rowptr, asm.col)
    vals = [asm.values(job.s, p) for p in job.p_list[:4]]
    h = pb.spai_build(job.s, job.p_list[0], approach="second")
    P1 = np_(h.export()["val"])
    Ps, qs = second_approach_diag(n, asm.rowptr, asm.col, vals, pat.P_rowptr, P1)
    scale = np.ones(n)
    for l in range(1, 4):
        h.update(job.s, job.p_list[l])
        exp = h.export()
        scale = scale * qs[l]
        np.testing.assert_allclose(np_(exp["q"]), scale, rtol=1e-13 * l)
        err = col_rel_err(n, pat.J_colptr, pat.P_slot, np_(exp["val"]), Ps[l])
        assert err <= 1e-12, (l, err)
    h.close()


def test_c1_adaptive_true_residual_every_point(c1):
    job, asm, pb, B = c1
    X, stats = pb.sequence_solve(B, [job.s] * len(job.p_list), job.p_list, policy="update",
                                 update="adaptive", adapt_ep=0.02)
    torch.cuda.synchronize()
    _check_residuals(job, asm, np_(X))
    assert all(st["cycles"] >= 1 and st["k"] == job.B.shape[1] for st in stats)
