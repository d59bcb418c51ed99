"""The adaptive Q pattern of the update (U-diag first, columns whose diagonal
misfit ||A(1)e_i - q_i A(l)e_i|| exceeds ep ||A(1)e_i|| escalated to the SPAI
pattern) on the GPU against the oracle.

Bars: Q within 1e-10 relative per column of the oracle's (ep placed in a gap of
the misfit ratios, so rounding cannot move a column across it), the update's
Frobenius misfit within 1e-9; block GMRES with Q P_1 reaches 1e-8 and matches
the oracle's run for the same steps with the GPU's preconditioner (1e-10); the
sequence path bit for bit the chain of single updates and solves.
"""
import numpy as np
import pytest
import torch

from synth import tiny_random_job
from oracle.assemble import Assembled
from oracle.spai import SpaiPattern
from oracle.update import diag_factors, update_adaptive
from oracle.gmres import block_gmres
from oracle.sparse import to_scipy
from oracle.sparse import transpose_pattern
from tests._helpers import np_, ctx as make_ctx, col_rel_err, gpu_P_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _ep_in_gap(n, asm, v1, vl):
    """an escalation threshold in the widest gap of the diagonal misfit ratios
    around their median (so that about half the columns escalate)"""
    q = diag_factors(n, asm.rowptr, asm.col, v1, vl)
    colptr, _, slot = transpose_pattern(n, asm.rowptr, asm.col)
    ratios = []
    for i in range(n):
        s = slot[colptr[i]:colptr[i + 1]]
        d = v1[s] - q[i] * vl[s]
        ratios.append(np.linalg.norm(d) / np.linalg.norm(v1[s]))
    r = np.sort(np.array(ratios))
    lo, hi = n // 4, 3 * n // 4
    k = lo + int(np.argmax(r[lo + 1:hi + 1] / np.maximum(r[lo:hi], 1e-300)))
    assert r[k + 1] > r[k] * (1 + 1e-6)
    return float(np.sqrt(r[k] * r[k + 1]))


def test_adaptive_update_matches_the_oracle_and_solves(ctx):
    from paper_1809_06574_amd import Problem
    job = tiny_random_job(300, 0.02, 81, k=2, npts=3)
    n = job.n
    asm = Assembled(job)
    pat = SpaiPattern(n, asm.rowptr, asm.col)
    v1, vl = asm.values(job.s, job.p_list[0]), asm.values(job.s, job.p_list[2])
    ep = _ep_in_gap(n, asm, v1, vl)
    qv, rho, esc = update_adaptive(n, asm.rowptr, asm.col, v1, vl, pat, ep)
    assert 0 < len(esc) < n
    pb = Problem(ctx, job.terms)
    h = pb.spai_build(job.s, job.p_list[0], update="adaptive", adapt_ep=ep)
    st = h.update(job.s, job.p_list[2], stats=True)
    exp = h.export()
    err = col_rel_err(n, pat.J_colptr, pat.P_slot, np_(exp["q"]), qv)
    assert err <= 1e-10, err
    assert st["fro_resid"] == pytest.approx(np.sqrt(np.sum(rho ** 2)), rel=1e-9)
    # block GMRES with Q P_1
    B = torch.as_tensor(job.B, device="cuda")
    X, sx, _ = pb.block_solve(h, job.s, job.p_list[2], B)
    A = to_scipy(n, asm.rowptr, asm.col, vl)
    Xg = np_(X)
    rel = np.linalg.norm(job.B - A @ Xg, axis=0) / np.linalg.norm(job.B, axis=0)
    assert np.all(rel <= 1e-8)
    Pf = gpu_P_apply(exp, n, "pattern", True)
    Xo, _ = block_gmres(A.__matmul__, Pf, job.B, m=30, tol=1e-8, fixed_steps=sx["cycle_steps"])
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) <= 1e-10
    h.close()
    pb.close()


def test_adaptive_sequence_equals_chain_of_single_updates(ctx):
    from paper_1809_06574_amd import Problem
    job = tiny_random_job(500, 0.005, 82, k=2, npts=5)
    n = job.n
    asm = Assembled(job)
    ep = _ep_in_gap(n, asm, asm.values(job.s, job.p_list[0]), asm.values(job.s, job.p_list[-1]))
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda")
    X, stats = pb.sequence_solve(B, [job.s] * len(job.p_list), job.p_list, policy="update", update="adaptive",
                                 adapt_ep=ep)
    h = pb.spai_build(job.s, job.p_list[0], update="adaptive", adapt_ep=ep)
    for l, p in enumerate(job.p_list):
        if l > 0:
            h.update(job.s, p)
        Xa, sa, _ = pb.block_solve(h, job.s, p, B)
        assert torch.equal(Xa, X[l]), l
        assert sa["cycle_steps"] == stats[l]["cycle_steps"]
    with pytest.raises(RuntimeError, match="adapt_ep"):
        pb.spai_build(job.s, job.p_list[0], update="adaptive", adapt_ep=-1.0)
    h.close()
    pb.close()


def test_adaptive_threshold_near_1e8(ctx):
    """p_l within 1e-7 of p_1: the diagonal misfit ratios are about 1e-8, where the
    expanded form of the residual would be rounding noise.  With ep in a gap of those
    ratios the escalated columns and Q are the oracle's (which forms a - q a_l)."""
    import dataclasses
    from paper_1809_06574_amd import Problem
    base = tiny_random_job(300, 0.02, 82, k=2, npts=3)
    p1 = float(base.p_list[0])
    job = dataclasses.replace(base, p_list=np.array([p1, p1 + 2e-7, p1 + 1e-7]))
    n = job.n
    asm = Assembled(job)
    pat = SpaiPattern(n, asm.rowptr, asm.col)
    v1, vl = asm.values(job.s, job.p_list[0]), asm.values(job.s, job.p_list[2])
    ep = _ep_in_gap(n, asm, v1, vl)
    assert 1e-10 < ep < 1e-6, ep
    qv, rho, esc = update_adaptive(n, asm.rowptr, asm.col, v1, vl, pat, ep)
    assert 0 < len(esc) < n
    pb = Problem(ctx, job.terms)
    h = pb.spai_build(job.s, job.p_list[0], update="adaptive", adapt_ep=ep)
    st = h.update(job.s, job.p_list[2], stats=True)
    exp = h.export()
    got = np_(exp["q"])
    err = col_rel_err(n, pat.J_colptr, pat.P_slot, got, qv)
    assert err <= 1e-10, err
    # the escalated set: a kept column has zeros off its diagonal
    rows = pat.J_row
    esc_gpu = []
    for i in range(n):
        sl = pat.P_slot[pat.J_colptr[i]:pat.J_colptr[i + 1]]
        off = rows[pat.J_colptr[i]:pat.J_colptr[i + 1]] != i
        if np.any(got[sl][off] != 0.0):
            esc_gpu.append(i)
    assert sorted(esc_gpu) == sorted(int(i) for i in esc)
    assert st["fro_resid"] == pytest.approx(np.sqrt(np.sum(rho ** 2)), rel=1e-6)
    h.close()
    pb.close()
