"""Batched solves: several independent systems in one lockstep block GMRES.

Each system of a batch must give bit for bit the X it gets when solved alone
(its sums depend on its own sizes only), every column must reach the 1e-8
relative residual, and the X must match the oracle's block GMRES run for the
same number of block steps with the GPU's preconditioner (1e-10 relative).
"""
import numpy as np
import pytest
import torch

from synth import config0, tiny_random_job
from synth.gen import _power_law_sizes, _nearest_pattern, _weighted_mdk, Job
from oracle.assemble import Assembled
from oracle.gmres import block_gmres
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx, gpu_P_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _residuals(job, s, p, X):
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(s, p))
    B = job.B
    nb = np.linalg.norm(B, axis=0)
    return np.linalg.norm(B - A @ X, axis=0) / np.where(nb > 0, nb, 1.0), A


def _oracle_parity(job, s, p, h, Xg, st, update_kind="diag", q_active=False, m=30):
    rel, A = _residuals(job, s, p, Xg)
    assert np.all(rel <= 1e-8), rel
    Pf = gpu_P_apply(h.export(), job.n, update_kind, q_active) if h is not None else (lambda X: X)
    Xo, _ = block_gmres(A.__matmul__, Pf, job.B, m=m, tol=1e-8, fixed_steps=st["cycle_steps"])
    d = np.linalg.norm(Xg - Xo) / max(np.linalg.norm(Xo), 1e-300)
    assert d <= 1e-10, (d, st)


def _systems(ctx):
    from paper_1809_06574_amd import Problem
    jobs = [tiny_random_job(300, 0.02, 11, k=2), config0(), tiny_random_job(515, 0.012, 12, k=2),
            tiny_random_job(129, 0.05, 13, k=2)]
    out = []
    for i, job in enumerate(jobs):
        pb = Problem(ctx, job.terms)
        upd = "pattern" if i == 2 else "diag"
        h = pb.spai_build(job.s, job.p_list[0], update=upd)
        p = job.p_list[1]
        if i != 3:
            h.update(job.s, p)
        out.append((job, pb, None if i == 3 else h, p, upd))
    return out


def test_batch_bitwise_equals_alone(ctx):
    from paper_1809_06574_amd import batch_solve
    sy = _systems(ctx)
    items = [(pb, h, job.s, p, torch.as_tensor(job.B, device="cuda")) for job, pb, h, p, _ in sy]
    Xs, stats, status, rc = batch_solve(ctx, items)
    assert rc == 0 and all(x == 0 for x in status)
    for (job, pb, h, p, upd), Xb, sb in zip(sy, Xs, stats):
        Xa, sa, _ = pb.block_solve(h, job.s, p, torch.as_tensor(job.B, device="cuda"))
        assert torch.equal(Xa, Xb), job.name
        assert sa["cycle_steps"] == sb["cycle_steps"]
        _oracle_parity(job, job.s, p, h, np_(Xb), sb, upd, q_active=(upd == "pattern"))


def test_batch_mixed_block_widths(ctx):
    """k = 1 and k = 3 systems share a kp = 4 batch; each matches its oracle."""
    from paper_1809_06574_amd import Problem, batch_solve
    jobs = [tiny_random_job(400, 0.015, 21, k=1), tiny_random_job(333, 0.02, 22, k=3)]
    items, hs = [], []
    for job in jobs:
        pb = Problem(ctx, job.terms)
        h = pb.spai_build(job.s, job.p_list[0])
        hs.append((pb, h))
        items.append((pb, h, job.s, job.p_list[0], torch.as_tensor(job.B, device="cuda")))
    Xs, stats, status, rc = batch_solve(ctx, items, m=20)
    assert rc == 0
    for job, (pb, h), X, st in zip(jobs, hs, Xs, stats):
        _oracle_parity(job, job.s, job.p_list[0], h, np_(X), st, m=20)


def test_batch_shared_problem_points(ctx):
    """Items of one problem at different points (the library assembles each)."""
    from paper_1809_06574_amd import Problem, batch_solve
    job = config0()
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    items = [(pb, None, job.s, p, B) for p in job.p_list]
    Xs, stats, status, rc = batch_solve(ctx, items)
    assert rc == 0
    for p, X, st in zip(job.p_list, Xs, stats):
        Xa, sa, _ = pb.block_solve(None, job.s, p, B)
        assert torch.equal(Xa, X)
        _oracle_parity(job, job.s, p, None, np_(X), st)


@pytest.mark.parametrize("policy,update", [("update", "diag"), ("update", "pattern"), ("rebuild", "diag")])
def test_sequence_batched_equals_pointwise(ctx, policy, update):
    from paper_1809_06574_amd import Problem
    job = tiny_random_job(600, 0.004, 31, k=2, npts=5)
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    s_list = [job.s] * len(job.p_list)
    X, stats = pb.sequence_solve(B, s_list, job.p_list, policy=policy, update=update)
    h = pb.spai_build(job.s, job.p_list[0], update=update)
    for l, p in enumerate(job.p_list):
        if l > 0:
            (h.update if policy == "update" else h.rebuild)(job.s, p)
        Xa, sa, _ = pb.block_solve(h, job.s, p, B)
        assert torch.equal(Xa, X[l]), (policy, update, l)
        assert sa["cycle_steps"] == stats[l]["cycle_steps"]
        rel, _ = _residuals(job, job.s, p, np_(X[l]))
        assert np.all(rel <= 1e-8)
        assert stats[l]["t_solve_ms"] > 0


def _power_law_system(i, dims):
    rng = np.random.default_rng([2024, i])
    terms = _weighted_mdk(dims, rng, 1e-3)
    K = terms["K0"]
    pat = _nearest_pattern(K, _power_law_sizes(rng, K.n))
    p = float(rng.uniform(0.1, 1.0))
    B = rng.standard_normal((K.n, 8))
    return Job(f"powerlaw_{i}", K.n, terms, 2.0, np.array([p, p + 0.02]), B, pattern=pat)


def test_batch_power_law_systems(ctx):
    """Systems of several sizes with power-law SPAI patterns, k = 8, in one batch;
    the update of each at its second point."""
    from paper_1809_06574_amd import Problem, batch_solve
    shapes = [(23, 17, 1), (9, 8, 6), (40, 31, 1), (7, 7, 7), (11, 10, 9), (30, 29, 1)]
    jobs = [_power_law_system(i, d) for i, d in enumerate(shapes)]
    sys_ = []
    for job in jobs:
        pb = Problem(ctx, job.terms)
        h = pb.spai_build(job.s, job.p_list[0], pattern=job.pattern)
        h.update(job.s, job.p_list[1])
        sys_.append((pb, h))
    items = [(pb, h, job.s, job.p_list[1], torch.as_tensor(job.B, device="cuda")) for job, (pb, h) in zip(jobs, sys_)]
    Xs, stats, status, rc = batch_solve(ctx, items)
    assert rc == 0
    for q, (job, (pb, h), X, st) in enumerate(zip(jobs, sys_, Xs, stats)):
        if q % 2 == 0:
            _oracle_parity(job, job.s, job.p_list[1], h, np_(X), st)
        else:
            rel, _ = _residuals(job, job.s, job.p_list[1], np_(X))
            assert np.all(rel <= 1e-8), rel
    # the same systems alone: bit for bit
    for (pb, h), job, X in zip(sys_[:2], jobs[:2], Xs[:2]):
        Xa, _, _ = pb.block_solve(h, job.s, job.p_list[1], torch.as_tensor(job.B, device="cuda"))
        assert torch.equal(Xa, X)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_spai_build_batch_equals_single_builds(ctx, precision):
    """spai_build_batch (the least squares of all systems in shared bucketed
    launches) gives every system bit for bit the P_1 of spai_build, for systems
    of the batch workload with explicit power-law patterns (every bucket, the
    LDS kernel included), a problem of roles and one problem at two points; an
    item with a bad point fails alone."""
    from paper_1809_06574_amd import Problem, spai_build_batch, lib as L
    from synth.gen import config2_system
    jobs = [config2_system(i) for i in (3, 17, 40)]
    pbs = [Problem(ctx, j.terms) for j in jobs]
    c0 = config0()
    pc0 = Problem(ctx, c0.terms)
    items = [(pb, j.s, j.p_list[0], j.pattern) for pb, j in zip(pbs, jobs)]
    items += [(pc0, c0.s, c0.p_list[0]), (pc0, c0.s, c0.p_list[2])]
    hs, status, rc = spai_build_batch(ctx, items, precision=precision)
    assert rc == 0 and all(x == 0 for x in status)
    for itm, h in zip(items, hs):
        pb, s, p = itm[:3]
        pat = itm[3] if len(itm) > 3 else None
        g = pb.spai_build(s, p, pattern=pat, precision=precision)
        e1, e2 = h.export(), g.export()
        for key in ("rowptr", "col", "val", "rho"):
            assert torch.equal(e1[key], e2[key]), key
        # the batched handle solves and updates like any other
        h.update(s, p + 0.02)
        g.update(s, p + 0.02)
        assert torch.equal(h.export()["val"], g.export()["val"])
    bad = list(items[:2]) + [(pbs[0], float("nan"), 0.5)]
    hs2, st2, rc2 = spai_build_batch(ctx, bad, precision=precision, raise_on_error=False)
    assert rc2 == L.PMOR_EINVAL and st2[:2] == [0, 0] and st2[2] == L.PMOR_EINVAL and hs2[2] is None
    fresh = pbs[0].spai_build(jobs[0].s, jobs[0].p_list[0], pattern=jobs[0].pattern, precision=precision)
    assert torch.equal(hs2[0].export()["val"], fresh.export()["val"])


def test_problem_create_batch_equals_single_creates(ctx):
    """pmor_problem_create_batch (union patterns built on worker streams) gives
    every problem bit for bit the pattern, maps and assembled values of the
    single create call, for problems of roles (the batch workload's systems and
    the 64^3-like job) and an affine one; a malformed item fails alone."""
    from paper_1809_06574_amd import Problem, problem_create_batch, lib as L
    from synth.gen import config2_system
    jobs = [config2_system(i) for i in (3, 17, 40, 41, 42, 43, 44, 45, 46, 47)]
    c0 = config0()
    aff = [c0.terms[r] for r in ("K0", "M0", "D0")]
    terms_list = [j.terms for j in jobs] + [c0.terms, aff]
    pbs, status, rc = problem_create_batch(ctx, terms_list)
    assert rc == 0 and all(x == 0 for x in status)
    for terms, pb in zip(terms_list, pbs):
        ref = Problem(ctx, terms)
        assert (pb.n, pb.nnz, pb.nmaps, pb.affine) == (ref.n, ref.nnz, ref.nmaps, ref.affine)
        for a, b in zip(pb.pattern(), ref.pattern()):
            assert torch.equal(a, b)
        pt = ([1.0, 0.25, 2.0], None) if pb.affine else (2.0, 0.4)
        assert torch.equal(pb.assemble(*pt), ref.assemble(*pt))
    # a problem from the batch builds, updates and solves like any other
    j = jobs[0]
    h = pbs[0].spai_build(j.s, j.p_list[0], pattern=j.pattern)
    h.update(j.s, j.p_list[1])
    X, st, rc1 = pbs[0].block_solve(h, j.s, j.p_list[1], torch.as_tensor(j.B, device="cuda"))
    assert rc1 == 0
    _oracle_parity(j, j.s, j.p_list[1], h, np_(X), st)
    # terms of different orders in one item: that item fails, the others are built
    bad = dict(jobs[1].terms)
    bad["K1"] = jobs[2].terms["K0"]
    pbs2, st2, rc2 = problem_create_batch(ctx, [jobs[0].terms, bad, aff], raise_on_error=False)
    assert rc2 == L.PMOR_EINVAL and st2 == [0, L.PMOR_EINVAL, 0] and pbs2[1] is None
    assert torch.equal(pbs2[0].pattern()[1], pbs[0].pattern()[1])
    # a column index out of range, found by the device validation on a worker stream
    K = jobs[3].terms["K0"]
    col = np.array(K.col, copy=True)
    col[5] = jobs[3].n + 7
    broken = dict(jobs[3].terms)
    broken["K0"] = (np.asarray(K.rowptr), col, np.asarray(K.val))
    pbs3, st3, rc3 = problem_create_batch(ctx, [aff, broken, jobs[4].terms], raise_on_error=False)
    assert rc3 == L.PMOR_EINVAL and st3 == [0, L.PMOR_EINVAL, 0] and pbs3[1] is None
    assert torch.equal(pbs3[2].pattern()[1], pbs[4].pattern()[1])


def test_spai_update_batch_equals_sequential_updates(ctx):
    """spai_update_batch leaves every handle bit for bit as spai_update does: the
    real U-diag updates queued together (first and second approach, FP32 and FP64
    least squares, two handles of one problem), a U-pattern handle and an affine
    problem's handle updated one after another; an item with a bad point fails
    alone."""
    from paper_1809_06574_amd import Problem, spai_update_batch, lib as L
    from synth.gen import config2_system
    jobs = [config2_system(i) for i in (5, 23)]
    c0 = config0()
    pbs = [Problem(ctx, j.terms) for j in jobs]
    p0 = Problem(ctx, c0.terms)
    aff = Problem(ctx, [c0.terms[r] for r in ("K0", "M0", "D0")])
    specs = [(pbs[0], jobs[0].s, jobs[0].p_list, dict(pattern=jobs[0].pattern, precision="f32")),
             (pbs[1], jobs[1].s, jobs[1].p_list, dict(pattern=jobs[1].pattern, approach="second")),
             (p0, c0.s, c0.p_list, dict()),
             (p0, c0.s, c0.p_list, dict(update="pattern")),
             (p0, c0.s, c0.p_list, dict(approach="second"))]

    def handles():
        hs = [pb.spai_build(s, pl[0], **kw) for pb, s, pl, kw in specs]
        hs.append(aff.spai_build([1.0, 0.5, 0.2], None))
        return hs

    ha, hb = handles(), handles()
    pts = [(s, pl[1]) for _, s, pl, _ in specs] + [([1.0, 0.6, 0.25], None)]
    for _ in range(2):  # two rounds: the second approach chains its anchor
        status, rc = spai_update_batch(ctx, [(h, *pt) for h, pt in zip(ha, pts)])
        assert rc == 0 and all(x == 0 for x in status)
        for h, pt in zip(hb, pts):
            h.update(*pt)
        for x, y in zip(ha, hb):
            ex, ey = x.export(), y.export()
            for key in ("val", "q", "rho"):
                assert torch.equal(ex[key], ey[key]), key
    st2, rc2 = spai_update_batch(ctx, [(ha[0], *pts[0]), (ha[2], float("nan"), 0.3), (ha[5], *pts[5])],
                                 raise_on_error=False)
    assert rc2 == L.PMOR_EINVAL and st2 == [0, L.PMOR_EINVAL, 0]
