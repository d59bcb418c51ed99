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
