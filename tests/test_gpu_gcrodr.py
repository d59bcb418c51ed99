"""Block GCRO-DR through the C ABI (block_solve_gcrodr, pmor_recycle_*) against
the oracle's block GCRO-DR replayed with the same block steps per cycle and the
library's preconditioner, along sequences of points (the recycled basis carried
from point to point, Section 3).

Bars: X within 1e-8 relative of the oracle at every point; the recycled
dimension equal to the oracle's and the recycled spans within 1e-6 (largest
principal angle); every true residual <= tol; with kr = 0 the cycles of block
GMRES (the engine's step counts, X within 1e-10 of the oracle's block GMRES).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import torch

from synth import config0, gyro_like_job, gyro_complex_job
from oracle.assemble import Assembled
from oracle.sparse import to_scipy
from oracle.gmres import block_gmres
from oracle.gcrodr import block_gcrodr
from oracle.complexsys import ComplexAssembled, real_form, complex_of
from tests._helpers import np_, ctx as make_ctx, gpu_P_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _resid(A, X, B):
    return np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)


def test_no_recycling_is_block_gmres(ctx):
    from paper_1809_06574_amd import Problem, Recycler
    job = config0()
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    p = job.p_list[1]
    h = pb.spai_build(job.s, p)
    B = torch.as_tensor(job.B, device="cuda")
    rec = Recycler(ctx, job.n, 0)
    X, st, rc = pb.block_solve_gcrodr(h, job.s, p, B, rec, m=6, tol=1e-10)
    assert rc == 0 and st["cycles"] >= 2 and rec.dim == 0
    _, st2, _ = pb.block_solve(h, job.s, p, B, m=6, tol=1e-10)
    assert st["cycle_steps"] == st2["cycle_steps"]
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
    Xo, _ = block_gmres(A.__matmul__, gpu_P_apply(h.export(), job.n), job.B, m=6, fixed_steps=st["cycle_steps"])
    assert _rel(np_(X), Xo) <= 1e-10
    assert np.all(_resid(A, np_(X), job.B) <= 1e-10)


def _sequence(ctx, pb, asm, values_at, pts, B_np, kr, m, tol, h_of=None, update="diag"):
    """GPU and oracle along the points; returns per-point GPU stats."""
    from paper_1809_06574_amd import Recycler
    n = B_np.shape[0]
    B = torch.as_tensor(B_np, device="cuda")
    rec = Recycler(ctx, n, kr)
    orc = {}
    h = None
    out = []
    for l, pt in enumerate(pts):
        if h_of is not None:
            if l == 0:
                h = h_of(pt)
            else:
                h.update(*pt)
        X, st, rc = pb.block_solve_gcrodr(h, *pt, B, rec, m=m, tol=tol)
        assert rc == 0, (l, rc)
        vals = values_at(pt)
        A = to_scipy(n, asm.rowptr, asm.col, vals)
        P = gpu_P_apply(h.export(), n, update, update == "pattern" and l > 0) if h is not None else (lambda Y: Y)
        Xo, io = block_gcrodr(A.__matmul__, P, B_np, m=m, kr=kr, fixed_steps=st["cycle_steps"], recycle=orc)
        Xg = np_(X)
        assert _rel(Xg, Xo) <= 1e-8, (l, _rel(Xg, Xo))
        assert np.all(_resid(A, Xg, B_np) <= tol), l
        Uo = orc["U"]
        assert rec.dim == (0 if Uo is None else Uo.shape[1]), l
        if rec.dim:
            assert sla.subspace_angles(np_(rec.export()), Uo).max() < 1e-6, l
        out.append(st)
    return out


def test_recycled_sequence_config0(ctx):
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pts = [(job.s, p) for p in job.p_list]
    sts = _sequence(ctx, pb, asm, lambda pt: asm.values(*pt), pts, job.B, kr=4, m=6, tol=1e-10,
                    h_of=lambda pt: pb.spai_build(*pt))
    assert all(s["cycles"] >= 1 for s in sts)


def test_recycled_sequence_nonsymmetric_gyroscope(ctx):
    """Complex harmonic Ritz values (non-symmetric A), kr large enough for pairs."""
    from paper_1809_06574_amd import Problem
    job = gyro_like_job(k=3)
    pb = Problem(ctx, [(T.rowptr, T.col, T.val) for T in job.aterms])
    asm = Assembled(job)
    pts = [(list(c), None) for c in job.coefs]
    _sequence(ctx, pb, asm, lambda pt: asm.values_c(pt[0]), pts, job.B, kr=7, m=5, tol=1e-10,
              h_of=lambda pt: pb.spai_build(*pt))


def test_unpreconditioned_and_pattern_update(ctx):
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pts = [(job.s, p) for p in job.p_list[:3]]
    _sequence(ctx, pb, asm, lambda pt: asm.values(*pt), pts, job.B, kr=4, m=10, tol=1e-9)
    _sequence(ctx, pb, asm, lambda pt: asm.values(*pt), pts, job.B, kr=4, m=5, tol=1e-10,
              h_of=lambda pt: pb.spai_build(*pt, update="pattern"), update="pattern")


def test_complex_points(ctx):
    """The complex gyroscope job in its real form: [R(B), R(iB)] solved with
    recycling along the points; the complex residuals."""
    from paper_1809_06574_amd import Problem, Recycler
    job = gyro_complex_job()
    pb = Problem(ctx, [(T.rowptr, T.col, T.val) for T in job.aterms], kinds=job.kinds)
    casm = ComplexAssembled(job)
    Bh = torch.as_tensor(np.hstack([real_form(job.B), real_form(1j * job.B)]), device="cuda")
    rec = Recycler(ctx, pb.n, 8)
    h = pb.spai_build(list(job.coefs[0]), None)
    steps = []
    for l, c in enumerate(job.coefs):
        if l:
            h.update(list(c))
        X, st, rc = pb.block_solve_gcrodr(h, list(c), None, Bh, rec, m=6, tol=1e-10)
        assert rc == 0
        A = sp.csr_matrix((casm.values(c), casm.col, casm.rowptr), shape=(job.n, job.n))
        Xc = complex_of(np_(X)[:, :job.k])
        assert np.all(_resid(A, Xc, job.B) <= 1e-9)
        steps.append(st["steps"])
    assert rec.dim > 0


def test_argument_errors(ctx):
    from paper_1809_06574_amd import Problem, Recycler, lib as L
    job = config0()
    pb = Problem(ctx, job.terms)
    B = torch.as_tensor(job.B, device="cuda").clone()
    rec = Recycler(ctx, job.n, 4)
    bad = Recycler(ctx, job.n + 1, 4)
    with pytest.raises(L.PmorError):
        pb.block_solve_gcrodr(None, job.s, 0.1, B, bad)
    B0 = B.clone()
    B0[:, 1] = 0.0
    with pytest.raises(L.PmorError):
        pb.block_solve_gcrodr(None, job.s, 0.1, B0, rec)
    with pytest.raises(L.PmorError):
        Recycler(ctx, job.n, 17)
    with pytest.raises(L.PmorError):
        pb.block_solve_gcrodr(None, job.s, 0.1, B, rec, m=0)
    # not converged within max_cycles
    X, st, rc = pb.block_solve_gcrodr(None, job.s, 0.1, B, rec, m=2, max_cycles=1, tol=1e-12,
                                      raise_on_error=False)
    assert rc == L.PMOR_ENOTCONV and st["cycles"] == 1
    rec.reset()
    assert rec.dim == 0


@pytest.mark.parametrize("k,kr,m", [(1, 16, 31), (16, 16, 3)])
def test_block_sizes_at_the_limits(ctx, k, kr, m):
    """One right-hand side with the largest recycled space and the longest
    cycle; sixteen right-hand sides (the largest block) with kr = 16: X against
    the oracle's replay at every point, equal recycled dimensions."""
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    B = np.random.default_rng(50 + k).standard_normal((job.n, k))
    pts = [(job.s, p) for p in job.p_list[:3]]
    _sequence(ctx, pb, asm, lambda pt: asm.values(*pt), pts, B, kr=kr, m=m, tol=1e-10,
              h_of=lambda pt: pb.spai_build(*pt))
