"""The C1 workload at its full size (64^3 grid, n = 262144, nnz(A) = 1,810,432,
k = 4, 20 points), solved as the benchmark solves it (pmor_sequence_solve, update
policy, all points together): exact checks where the oracle is cheap at this size
(union pattern and slot maps, index sets, U-diag factors), the true residual of
every point, and SPAI columns sampled where the oracle solves them one by one."""
import numpy as np
import pytest
import torch

from synth import config1
from oracle.assemble import Assembled
from oracle.spai import pattern_of_A, shadow, solve_column
from oracle.sparse import to_scipy, transpose_pattern
from oracle.update import diag_factors
from tests._helpers import np_

pytestmark = pytest.mark.gpu


class _Sets:
    """J_j and I_j of the oracle, in the form solve_column reads."""

    def __init__(self, jc, jr, ic, ir):
        self.jc, self.jr, self.ic, self.ir = jc, jr, ic, ir

    def J(self, j):
        return self.jr[self.jc[j]:self.jc[j + 1]]

    def I(self, j):
        return self.ir[self.ic[j]:self.ic[j + 1]]


@pytest.fixture(scope="module")
def c1(gpu_lib):
    from paper_1809_06574_amd import Context, Problem
    job = config1()
    asm = Assembled(job)
    ctx = Context(0)
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    X, stats = pb.sequence_solve(B, [job.s] * len(job.p_list), job.p_list, policy="update")
    torch.cuda.synchronize()
    yield job, asm, pb, np_(X), stats
    pb.close()
    ctx.close()


def test_c1_shape(c1):
    job, asm, pb, X, stats = c1
    assert job.n == 262144 and asm.nnz == 1810432 and len(job.p_list) == 20 and job.B.shape[1] == 4


def test_c1_union_pattern_and_maps_bitexact(c1):
    job, asm, pb, X, stats = c1
    rp, ci, mp = pb.pattern()
    np.testing.assert_array_equal(np_(rp), asm.rowptr)
    np.testing.assert_array_equal(np_(ci), asm.col)
    for r, role in enumerate(("M0", "M1", "D0", "D1", "K0", "K1")):
        want = asm.maps.get(role, np.full(asm.nnz, -1, dtype=np.int32))
        np.testing.assert_array_equal(np_(mp[r]), want, err_msg=role)


def test_c1_true_residual_every_point(c1):
    job, asm, pb, X, stats = c1
    bn = np.linalg.norm(job.B, axis=0)
    for l, p in enumerate(job.p_list):
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
        rel = np.linalg.norm(job.B - A @ X[l], axis=0) / bn
        assert np.all(rel <= 1e-8 * 1.0001), (l, rel)
        assert stats[l]["cycles"] >= 1


def test_c1_index_sets_and_sampled_spai_columns(c1):
    job, asm, pb, X, stats = c1
    n = job.n
    h = pb.spai_build(job.s, job.p_list[0])
    jc, jr, ic, ir = h.export_sets()
    ojc, ojr = pattern_of_A(n, asm.rowptr, asm.col)
    oic, oir = shadow(n, ojc, ojr, asm.rowptr, asm.col)
    np.testing.assert_array_equal(np_(jc), ojc)
    np.testing.assert_array_equal(np_(jr), ojr)
    np.testing.assert_array_equal(np_(ic), oic)
    np.testing.assert_array_equal(np_(ir), oir)
    # columns: the grid's corners, edges and faces, and random interior ones
    rng = np.random.default_rng(2026)
    cols = np.unique(np.concatenate([[0, 63, 4095, 4096 * 63, n - 1], rng.integers(0, n, 160)]))
    exp = h.export()
    prp, pci, pv = np_(exp["rowptr"]), np_(exp["col"]), np_(exp["val"])
    pcp, prow, pslot = transpose_pattern(n, prp, pci)
    val = asm.values(job.s, job.p_list[0])
    sets = _Sets(ojc, ojr, oic, oir)
    worst = 0.0
    for j in cols:
        x, rho = solve_column(n, asm.rowptr, asm.col, val, sets, int(j))
        np.testing.assert_array_equal(prow[pcp[j]:pcp[j + 1]], sets.J(int(j)))
        got = pv[pslot[pcp[j]:pcp[j + 1]]]
        worst = max(worst, np.linalg.norm(got - x) / np.linalg.norm(x))
    assert worst <= 1e-10, worst
    h.close()


@pytest.mark.parametrize("l", [1, 10, 19])
def test_c1_update_factors_every_column(c1, l):
    job, asm, pb, X, stats = c1
    h = pb.spai_build(job.s, job.p_list[0])
    h.update(job.s, job.p_list[l])
    q = np_(h.export()["q"])
    want = diag_factors(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[0]),
                        asm.values(job.s, job.p_list[l]))
    rel = np.max(np.abs(q - want) / np.abs(want))
    assert rel <= 1e-13, rel
    h.close()


@pytest.fixture(scope="module")
def c2(gpu_lib):
    """Six systems of the batch workload at their full sizes, prepared and solved
    together as the benchmark does (P_1 at p, U-diag update at p + 0.02,
    pmor_batch_solve)."""
    from synth.gen import config2_system
    from paper_1809_06574_amd import Context, Problem, batch_solve
    jobs = [config2_system(i) for i in range(6)]
    ctx = Context(0)
    pbs, hs, Bs = [], [], []
    for job in jobs:
        pb = Problem(ctx, job.terms)
        h = pb.spai_build(job.s, job.p_list[0], pattern=job.pattern)
        h.update(job.s, job.p_list[1])
        pbs.append(pb)
        hs.append(h)
        Bs.append(torch.as_tensor(job.B, device="cuda"))
    items = [(pb, h, job.s, job.p_list[1], B) for pb, h, job, B in zip(pbs, hs, jobs, Bs)]
    Xs, stats, status, rc = batch_solve(ctx, items)
    torch.cuda.synchronize()
    yield jobs, pbs, hs, [np_(X) for X in Xs], status
    for h in hs:
        h.close()
    for pb in pbs:
        pb.close()
    ctx.close()


def test_c2_true_residuals(c2):
    jobs, pbs, hs, Xs, status = c2
    assert all(s == 0 for s in status)
    for job, X in zip(jobs, Xs):
        asm = Assembled(job)
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[1]))
        rel = np.linalg.norm(job.B - A @ X, axis=0) / np.linalg.norm(job.B, axis=0)
        assert np.all(rel <= 1e-8 * 1.0001), (job.name, rel)


def test_c2_shadows_and_sampled_anchor_columns(c2):
    jobs, pbs, hs, Xs, status = c2
    rng = np.random.default_rng(2027)
    for job, pb in zip(jobs[:3], pbs[:3]):
        n = job.n
        asm = Assembled(job)
        h = pb.spai_build(job.s, job.p_list[0], pattern=job.pattern)  # P_1 (the update overwrote the other)
        jc, jr, ic, ir = h.export_sets()
        ojc, ojr = job.pattern
        oic, oir = shadow(n, ojc, ojr, asm.rowptr, asm.col)
        np.testing.assert_array_equal(np_(ic), oic)
        np.testing.assert_array_equal(np_(ir), oir)
        exp = h.export()
        pcp, prow, pslot = transpose_pattern(n, np_(exp["rowptr"]), np_(exp["col"]))
        pv = np_(exp["val"])
        val = asm.values(job.s, job.p_list[0])
        sets = _Sets(np.asarray(ojc), np.asarray(ojr), oic, oir)
        lens = np.diff(np.asarray(ojc))
        cols = np.unique(np.concatenate([np.flatnonzero(lens == lens.max())[:8], rng.integers(0, n, 40)]))
        worst = 0.0
        for j in cols:
            x, rho = solve_column(n, asm.rowptr, asm.col, val, sets, int(j))
            np.testing.assert_array_equal(prow[pcp[j]:pcp[j + 1]], sets.J(int(j)))
            got = pv[pslot[pcp[j]:pcp[j + 1]]]
            worst = max(worst, np.linalg.norm(got - x) / np.linalg.norm(x))
        assert worst <= 1e-10, (job.name, worst)
        h.close()


def test_c4_largest_job_served_with_a_small_one(gpu_lib):
    """The serving workload's largest size class (128 x 128 x 64, n = 1,048,576,
    20 points) served together with a small job, as in the benchmark's mix:
    every point of both at relative residual <= 1e-8."""
    from synth.gen import config4_job
    from paper_1809_06574_amd import Context, Problem, Server
    jobs = [config4_job(0, size_class=3), config4_job(1, size_class=0)]
    assert jobs[0].n == 1048576
    ctx = Context(0)
    sv = Server(ctx, k=4)
    pbs = [Problem(ctx, j.terms) for j in jobs]
    Bs = [torch.as_tensor(j.B, device="cuda") for j in jobs]
    ids = {sv.submit(pb, B, [j.s] * len(j.p_list), j.p_list): q for q, (pb, B, j) in enumerate(zip(pbs, Bs, jobs))}
    out, steps = {}, 0
    while len(out) < len(jobs):
        for jid, status, X, stats in sv.step():
            out[ids[jid]] = (status, np_(X))
        steps += 1
        assert steps < 10000
    sv.close()
    for q, job in enumerate(jobs):
        status, X = out[q]
        assert status == 0
        asm = Assembled(job)
        bn = np.linalg.norm(job.B, axis=0)
        for l, p in enumerate(job.p_list):
            A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
            rel = np.linalg.norm(job.B - A @ X[l], axis=0) / bn
            assert np.all(rel <= 1e-8 * 1.0001), (job.name, l, rel)
    for pb in pbs:
        pb.close()
    ctx.close()
