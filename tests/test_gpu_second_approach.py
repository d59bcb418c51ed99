"""The second update approach of Table 1 (anchor A(l-1), P_l = Q_l P_{l-1}),
U-diag reading, on the GPU against the oracle's chain.

Bars: the running row scale and P_l within 1e-12 relative of the oracle's
literal chain (the library keeps P_l = diag(q_l ... q_2) P_1, the oracle forms
diag(q_l) P_{l-1}: the same factors in another rounding order); the sequence
path (all points' factors in chained launches) bit for bit the X of a chain of
single updates and solves; every column at relative residual <= 1e-8.
"""
import numpy as np
import pytest
import torch

from synth import config0, tiny_random_job
from oracle.assemble import Assembled
from oracle.spai import SpaiPattern
from oracle.update import diag_factors, second_approach_diag
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx, col_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _residuals(job, s, p, X):
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(s, p))
    nb = np.linalg.norm(job.B, axis=0)
    return np.linalg.norm(job.B - A @ X, axis=0) / np.where(nb > 0, nb, 1.0)


@pytest.mark.parametrize("which", ["config0", "tiny"])
def test_handle_chain_matches_the_oracle(ctx, which):
    from paper_1809_06574_amd import Problem
    job = config0() if which == "config0" else tiny_random_job(90, 0.05, 61, npts=6)
    n = job.n
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(n, asm.rowptr, asm.col)
    vals = [asm.values(job.s, p) for p in job.p_list]
    h = pb.spai_build(job.s, job.p_list[0], approach="second")
    P1 = np_(h.export()["val"])  # the library's P_1 is the chain's input
    Ps, qs = second_approach_diag(n, asm.rowptr, asm.col, vals, pat.P_rowptr, P1)
    scale = np.ones(n)
    for l in range(1, len(job.p_list)):
        h.update(job.s, job.p_list[l])
        exp = h.export()
        scale = scale * qs[l]
        np.testing.assert_allclose(np_(exp["q"]), scale, rtol=1e-13 * l)
        err = col_rel_err(n, pat.J_colptr, pat.P_slot, np_(exp["val"]), Ps[l])
        assert err <= 1e-12, (l, err)
        # the step's own residual ||A(l-1) e_i - q_i A(l) e_i||
        Aprev = to_scipy(n, asm.rowptr, asm.col, vals[l - 1]).toarray()
        Al = to_scipy(n, asm.rowptr, asm.col, vals[l]).toarray()
        rho = np.linalg.norm(Aprev - Al * qs[l][None, :], axis=0)
        # (the library forms rho^2 = |a|^2 - 2 q <a, A(l) e_i> + q^2 |A(l) e_i|^2: sqrt(eps)-level absolute error)
        np.testing.assert_allclose(np_(exp["rho"]), rho, rtol=1e-9, atol=1e-6 * np.abs(Aprev).max())
    # the first update of the chain is the first approach's update
    h2 = pb.spai_build(job.s, job.p_list[0])
    h2.update(job.s, job.p_list[1])
    h3 = pb.spai_build(job.s, job.p_list[0], approach="second")
    h3.update(job.s, job.p_list[1])
    assert torch.equal(h2.export()["val"], h3.export()["val"])
    # a rebuild re-anchors: the next update is again against the rebuilt point
    h.rebuild(job.s, job.p_list[1])
    h.update(job.s, job.p_list[2])
    q = diag_factors(n, asm.rowptr, asm.col, vals[1], vals[2])
    np.testing.assert_allclose(np_(h.export()["q"]), q, rtol=1e-13)
    for x in (h, h2, h3):
        x.close()
    pb.close()


def test_sequence_equals_chain_of_single_updates(ctx):
    """11 points: the factors of points 1..10 take two chained launches (8 per
    launch), the running scale carried between them."""
    from paper_1809_06574_amd import Problem
    job = tiny_random_job(500, 0.005, 62, k=2, npts=11)
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    s_list = [job.s] * len(job.p_list)
    X, stats = pb.sequence_solve(B, s_list, job.p_list, policy="update", approach="second")
    h = pb.spai_build(job.s, job.p_list[0], approach="second")
    for l, p in enumerate(job.p_list):
        if l > 0:
            h.update(job.s, p)
        Xa, sa, _ = pb.block_solve(h, job.s, p, B)
        assert torch.equal(Xa, X[l]), l
        assert sa["cycle_steps"] == stats[l]["cycle_steps"]
        assert np.all(_residuals(job, job.s, p, np_(X[l])) <= 1e-8)
    h.close()
    pb.close()


def test_second_approach_needs_the_diag_update(ctx):
    from paper_1809_06574_amd import Problem
    job = tiny_random_job(40, 0.1, 63)
    pb = Problem(ctx, job.terms)
    with pytest.raises(RuntimeError, match="second update approach"):
        pb.spai_build(job.s, job.p_list[0], update="pattern", approach="second")
    pb.close()
