"""Block GMRES on the GPU against the oracle in the configurations the ordinary
solves do not reach: full 30-step cycles followed by a restart (every register
size of the Gram-Schmidt kernels), dependent right-hand-side columns, and a
column whose Krylov space stops growing long before the others converge.

Bars: X within 1e-10 relative of the oracle replaying the GPU's block steps per
cycle; the verdict (converged, not converged, breakdown) equal to the oracle's.
"""
import dataclasses

import numpy as np
import pytest
import torch

from synth import config0, config1
from oracle.assemble import Assembled
from oracle.gmres import block_gmres
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx, gpu_P_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _ident(X):
    return X


def _replay(job, A, Pf, B, Xg, st, m, tol):
    Xo, info = block_gmres(A.__matmul__, Pf, B, m=m, tol=tol, fixed_steps=st["cycle_steps"])
    d = np.linalg.norm(Xg - Xo) / max(np.linalg.norm(Xo), 1e-300)
    return d, info


@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
def test_full_cycles_then_restart(ctx, k):
    """A 16^3 weighted Laplacian with s = 0.05 (A close to K, condition number about
    1e3) and no preconditioner: two cycles of 30 block steps never reach tol 1e-14,
    so every sweep length 1..30 of the Gram-Schmidt passes runs (register counts
    NB = 4..32 at kp = 4, 1..4 or 2..8 blocks per wavefront at kp = 1, 2, 8, 16),
    the second cycle after a restart."""
    from paper_1809_06574_amd import Problem
    from paper_1809_06574_amd import lib as L
    job = dataclasses.replace(config1(dims=(16, 16, 16), npts=1, k=k, seed=5100 + k), s=0.05)
    pb = Problem(ctx, job.terms)
    p = job.p_list[0]
    B = torch.as_tensor(job.B, device="cuda")
    X, st, rc = pb.block_solve(None, job.s, p, B, m=30, tol=1e-14, max_cycles=2, raise_on_error=False)
    assert rc == L.PMOR_ENOTCONV
    assert st["cycles"] == 2 and st["cycle_steps"] == [30, 30], st
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
    d, info = _replay(job, A, _ident, job.B, np_(X), st, 30, 1e-14)
    assert d <= 1e-10, d
    # the reported residuals are the true ones
    rel = np.linalg.norm(job.B - A @ np_(X), axis=0) / np.linalg.norm(job.B, axis=0)
    np.testing.assert_allclose(st["relres"][:k], rel, rtol=1e-6)


def test_full_cycles_then_restart_preconditioned(ctx):
    """The same sweep lengths with the SPAI preconditioner, updated (U-diag), at k = 4
    and k = 16; the solve converges after the restart."""
    from paper_1809_06574_amd import Problem
    for k in (4, 16):
        job = dataclasses.replace(config1(dims=(16, 16, 16), npts=2, k=k, seed=5200 + k), s=0.05)
        pb = Problem(ctx, job.terms)
        h = pb.spai_build(job.s, job.p_list[0])
        h.update(job.s, job.p_list[1])
        p = job.p_list[1]
        B = torch.as_tensor(job.B, device="cuda")
        X, st, rc = pb.block_solve(h, job.s, p, B, m=30, tol=1e-13, max_cycles=20)
        assert st["cycles"] >= 2 and st["cycle_steps"][0] == 30, st
        asm = Assembled(job)
        A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
        Pf = gpu_P_apply(h.export(), job.n)
        d, _ = _replay(job, A, Pf, job.B, np_(X), st, 30, 1e-13)
        assert d <= 1e-10, (k, d)
        rel = np.linalg.norm(job.B - A @ np_(X), axis=0) / np.linalg.norm(job.B, axis=0)
        assert np.all(rel <= 1e-13 * 1.0001), rel


@pytest.mark.parametrize("eps", [0.0, 1e-10, 1e-3])
@pytest.mark.parametrize("precond", [False, True])
def test_dependent_rhs_columns(ctx, eps, precond):
    """b_2 = b_1 + eps-sized noise.  eps = 0 and 1e-10: the residual block at the first
    cycle start is dependent, the GPU returns PMOR_EBREAKDOWN with X = 0 after a
    cycle of no steps, as the oracle does.  eps = 1e-3: both converge and agree."""
    from paper_1809_06574_amd import Problem
    from paper_1809_06574_amd import lib as L
    job = config0()
    pb = Problem(ctx, job.terms)
    p = job.p_list[0]
    h = pb.spai_build(job.s, p) if precond else None
    rng = np.random.default_rng(77)
    b = job.B[:, 0]
    Bh = np.column_stack([b, b + eps * np.linalg.norm(b) * rng.standard_normal(job.n) / np.sqrt(job.n)])
    X, st, rc = pb.block_solve(h, job.s, p, torch.as_tensor(Bh, device="cuda"), raise_on_error=False)
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
    Pf = gpu_P_apply(h.export(), job.n) if precond else _ident
    Xo, info = block_gmres(A.__matmul__, Pf, Bh, m=30, tol=1e-8)
    if eps < 1e-6:
        assert info.breakdown and info.steps == [0]
        assert rc == L.PMOR_EBREAKDOWN, rc
        assert st["cycles"] == 1 and st["cycle_steps"] == [0]
        assert not np_(X).any()
    else:
        assert info.converged and rc == 0
        d, _ = _replay(job, A, Pf, Bh, np_(X), st, 30, 1e-8)
        assert d <= 1e-10, d


@pytest.mark.parametrize("noise", [0.0, 1e-11])
def test_column_with_small_krylov_space(ctx, noise):
    """b_1 is a combination of two eigenvectors of the symmetric C0 matrix (noise = 0),
    or that plus noise of relative size 1e-11, so b_1 is solved (to about the noise)
    by the second block step, long before b_2 and b_3.  noise = 0: the block stops
    growing there, and GPU and oracle both end the first cycle after 2 steps, restart
    and converge.  noise = 1e-11: the new block keeps a column of relative size 1e-11
    in a direction of its own (not a dependent one), so both run on; the verdicts and
    first cycles' step counts agree and X matches."""
    from paper_1809_06574_amd import Problem
    job = config0(k=3)
    pb = Problem(ctx, job.terms)
    p = job.p_list[0]
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
    w, U = np.linalg.eigh(A.toarray())
    rng = np.random.default_rng(5)
    b1 = U[:, 3] + 0.5 * U[:, 700]
    b1 = b1 + noise * np.linalg.norm(b1) * rng.standard_normal(job.n) / np.sqrt(job.n)
    Bh = np.column_stack([b1, job.B[:, 1], job.B[:, 2]])
    X, st, rc = pb.block_solve(None, job.s, p, torch.as_tensor(Bh, device="cuda"), tol=1e-10)
    Xo, info = block_gmres(A.__matmul__, _ident, Bh, m=30, tol=1e-10)
    assert info.converged and rc == 0
    assert st["cycle_steps"][0] == info.steps[0], (st, info.steps)
    if noise == 0.0:
        assert info.steps[0] == 2
    d, _ = _replay(job, A, _ident, Bh, np_(X), st, 30, 1e-10)
    assert d <= 1e-10, d
    rel = np.linalg.norm(Bh - A @ np_(X), axis=0) / np.linalg.norm(Bh, axis=0)
    assert np.all(rel <= 1e-10 * 1.0001), rel
