"""Re-anchoring of a sequence (first approach, U-diag): a point whose update
misfit ||A(a) - A(l) diag(q)||_F / ||A(a)||_F against the current anchor a
exceeds the tolerance gets a fresh SPAI and anchors the later points.

Bars: the anchors equal the oracle's plan (tolerance placed in a wide gap of
the misfits, so rounding cannot move a decision); each run between anchors is
bit for bit the same sequence solved on its own; every column at relative
residual <= 1e-8; the unsupported combinations are rejected.
"""
import numpy as np
import pytest
import torch

from synth import tiny_random_job
from oracle.assemble import Assembled
from oracle.update import misfit_diag, plan_anchors
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx

pytestmark = pytest.mark.gpu

PS = [0.05, 0.06, 0.07, 0.5, 0.51, 0.52, 0.95, 0.96, 0.97, 0.98]


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _job():
    return tiny_random_job(400, 0.01, 71, k=2, npts=len(PS))


def _tol_and_plan(job):
    asm = Assembled(job)
    vals = [asm.values(job.s, p) for p in PS]
    n = job.n
    close = [misfit_diag(n, asm.rowptr, asm.col, vals[a], vals[b])
             for a, b in ((0, 1), (0, 2), (3, 4), (3, 5), (6, 7), (6, 8), (6, 9))]
    far = [misfit_diag(n, asm.rowptr, asm.col, vals[0], vals[3]), misfit_diag(n, asm.rowptr, asm.col, vals[3], vals[6])]
    assert min(far) > 10 * max(close)
    tol = float(np.sqrt(min(far) * max(close)))
    return tol, plan_anchors(n, asm.rowptr, asm.col, vals, tol), asm


def test_anchors_match_the_oracle_and_runs_are_sequences(ctx):
    from paper_1809_06574_amd import Problem
    job = _job()
    tol, plan, asm = _tol_and_plan(job)
    assert plan == [0, 3, 6]
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    X, st = pb.sequence_solve(B, [job.s] * len(PS), PS, policy="update", reanchor_tol=tol)
    anchors = [s["anchor"] for s in st]
    assert anchors == [0, 0, 0, 3, 3, 3, 6, 6, 6, 6]
    bounds = plan + [len(PS)]
    for a, b in zip(bounds[:-1], bounds[1:]):
        Xr, sr = pb.sequence_solve(B, [job.s] * (b - a), PS[a:b], policy="update")
        for t in range(b - a):
            assert torch.equal(Xr[t], X[a + t]), (a, t)
            assert sr[t]["cycle_steps"] == st[a + t]["cycle_steps"]
            if t > 0:  # the update misfit against the run's own anchor
                rel = st[a + t]["fro_resid"] / np.linalg.norm(asm.values(job.s, PS[a]))
                assert rel <= tol
    for l, p in enumerate(PS):
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
        r = np.linalg.norm(job.B - A @ np_(X[l]), axis=0) / np.linalg.norm(job.B, axis=0)
        assert np.all(r <= 1e-8), (l, r)
    # a tolerance above every misfit keeps the single anchor
    X1, s1 = pb.sequence_solve(B, [job.s] * len(PS), PS, policy="update", reanchor_tol=1e6)
    X0, s0 = pb.sequence_solve(B, [job.s] * len(PS), PS, policy="update")
    assert torch.equal(X1, X0) and all(s["anchor"] == 0 for s in s1)
    pb.close()


def test_reanchoring_rejected_where_not_built(ctx):
    from paper_1809_06574_amd import Problem
    job = tiny_random_job(60, 0.05, 72, k=2, npts=3)
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    sl = [job.s] * 3
    for kw in ({"policy": "rebuild"}, {"update": "pattern"}, {"approach": "second"}):
        args = dict(policy="update", reanchor_tol=0.1)
        args.update(kw)
        with pytest.raises(RuntimeError, match="re-anchoring"):
            pb.sequence_solve(B, sl, list(job.p_list), **args)
    with pytest.raises(RuntimeError, match="reanchor_tol"):
        pb.sequence_solve(B, sl, list(job.p_list), policy="update", reanchor_tol=-1.0)
    pb.close()
