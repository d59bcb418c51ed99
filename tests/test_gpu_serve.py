"""Serving: sequence jobs admitted under a memory budget, their points solved
in one persistent engine with continuous batching (systems join and leave at
restart-cycle boundaries).

A job's X must not depend on what else shares the engine: bit for bit the X of
the same job served alone and of pmor_sequence_solve (same block width), and
every point at relative residual <= 1e-8.
"""
import numpy as np
import pytest
import torch

from synth.gen import _weighted_mdk, Job
from oracle.assemble import Assembled
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx

pytestmark = pytest.mark.gpu

DIMS = ((8, 8, 4), (16, 8, 8), (12, 12, 12), (24, 16, 8), (10, 9, 7), (20, 20, 6))


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _job(jid, npts=6, k=4):
    rng = np.random.default_rng([1004, 777, jid])
    dims = DIMS[jid % len(DIMS)]
    terms = _weighted_mdk(dims, rng, 1e-3)
    n = terms["K0"].n
    p0 = float(rng.uniform(0.1, 0.6))
    B = rng.standard_normal((n, k))
    return Job(f"serve_{jid}", n, terms, 2.0, p0 + 0.02 * np.arange(npts), B, meta={"dims": dims})


def _serve(ctx, jobs, submit_at, policy="update", **kw):
    """Run a server; job q is submitted before step submit_at[q].  Returns {q: (status, X, stats)}."""
    from paper_1809_06574_amd import Problem, Server
    sv = Server(ctx, k=4, **kw)
    pbs = [Problem(ctx, j.terms) for j in jobs]
    Bs = [torch.as_tensor(j.B, device="cuda") for j in jobs]
    ids, out, step = {}, {}, 0
    while len(out) < len(jobs):
        for q, j in enumerate(jobs):
            if submit_at[q] == step:
                ids[sv.submit(pbs[q], Bs[q], [j.s] * len(j.p_list), j.p_list, policy=policy)] = q
        for jid, status, X, stats in sv.step():
            out[ids[jid]] = (status, X.clone(), stats)
        step += 1
        assert step < 10000
    info = sv.info()
    assert info["queued"] == 0 and info["admitted"] == 0 and info["running"] == 0
    sv.close()
    return out


def _check_residuals(job, X):
    asm = Assembled(job)
    for l, p in enumerate(job.p_list):
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
        rel = np.linalg.norm(job.B - A @ np_(X[l]), axis=0) / np.linalg.norm(job.B, axis=0)
        assert np.all(rel <= 1e-8), (job.name, l, rel)


@pytest.mark.parametrize("policy", ["update", "rebuild"])
def test_served_alone_vs_in_the_mix_bitwise(ctx, policy):
    from paper_1809_06574_amd import Problem
    jobs = [_job(q) for q in range(6)]
    mix = _serve(ctx, jobs, submit_at=[0, 0, 1, 3, 4, 9], policy=policy, max_systems=12)
    for q, job in enumerate(jobs):
        status, X, stats = mix[q]
        assert status == 0, (q, status)
        _check_residuals(job, X)
        assert all(s["t_solve_ms"] > 0 for s in stats)
    for q in (0, 3, 5):
        alone = _serve(ctx, [jobs[q]], submit_at=[0], policy=policy, max_systems=12)
        assert torch.equal(alone[0][1], mix[q][1]), q
        pb = Problem(ctx, jobs[q].terms)
        B = torch.as_tensor(jobs[q].B, device="cuda")
        Xs, _ = pb.sequence_solve(B, [jobs[q].s] * len(jobs[q].p_list), jobs[q].p_list, policy=policy)
        assert torch.equal(Xs, mix[q][1]), q


def test_budget_admits_one_job_at_a_time(ctx):
    """A budget that holds the engine and one job but not two: jobs are served
    in order, one at a time, and a job that can never fit is refused."""
    from paper_1809_06574_amd import Problem, Server, lib as L
    jobs = [_job(q, npts=3) for q in (3, 9, 15)]  # the same grid size, different seeds
    pbs = [Problem(ctx, j.terms) for j in jobs]
    Bs = [torch.as_tensor(j.B, device="cuda") for j in jobs]
    # footprint of one job: bytes held with it admitted minus the engine's
    probe = Server(ctx, k=4, engine_rows=8192, max_systems=8)
    eng = probe.info()["bytes"]
    probe.submit(pbs[0], Bs[0], [jobs[0].s] * 3, jobs[0].p_list)
    probe.step()
    foot = probe.info()["bytes"] - eng
    while probe.info()["admitted"]:
        probe.step()
    probe.close()
    assert foot > 0
    sv = Server(ctx, k=4, hbm_budget=eng + foot + foot // 2, engine_rows=8192, max_systems=8)
    ids = [sv.submit(pb, B, [j.s] * 3, j.p_list) for pb, B, j in zip(pbs, Bs, jobs)]
    seen_admitted, order, Xs = 0, [], {}
    while len(order) < len(jobs):
        for jid, status, X, stats in sv.step():
            assert status == 0
            order.append(jid)
            Xs[jid] = X.clone()
        seen_admitted = max(seen_admitted, sv.info()["admitted"])
    assert order == ids
    assert seen_admitted == 1
    for jid, job in zip(ids, jobs):
        _check_residuals(job, Xs[jid])
    terms = _weighted_mdk((64, 64, 32), np.random.default_rng(5), 1e-3)
    pb_big = Problem(ctx, terms)
    Bb = torch.ones((terms["K0"].n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(L.PmorError) as e:
        sv.submit(pb_big, Bb, [2.0] * 3, [0.1, 0.2, 0.3])
    assert e.value.code == L.PMOR_EADMIT
    sv.close()


@pytest.mark.parametrize("kind", [{"update": "pattern"}, {"update": "adaptive", "adapt_ep": 0.02},
                                  {"approach": "second"}])
def test_served_update_variants_match_sequence_solve(ctx, kind):
    """The U-pattern and adaptive updates and the second approach through the
    server: every job bit for bit its pmor_sequence_solve result."""
    from paper_1809_06574_amd import Problem
    jobs = [_job(q) for q in (1, 2, 4)]
    mix = _serve(ctx, jobs, submit_at=[0, 0, 2], policy="update", max_systems=12, **kind)
    for q, job in enumerate(jobs):
        status, X, stats = mix[q]
        assert status == 0, (q, status)
        _check_residuals(job, X)
        pb = Problem(ctx, job.terms)
        B = torch.as_tensor(job.B, device="cuda")
        Xs, _ = pb.sequence_solve(B, [job.s] * len(job.p_list), job.p_list, policy="update", **kind)
        assert torch.equal(Xs, X), (q, kind)
        pb.close()
