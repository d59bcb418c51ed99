"""The general affine problem A(c) = sum_t c_t T_t (Section 1.1, eq. affine_system;
Section 2.4) and the import of a given preconditioner, through the C ABI, against
the oracle on a job shaped like the paper's gyroscope model (seven terms, six free
coefficients, non-symmetric).

Bars: union pattern and slot maps bit-exact; assembly within 8 eps of the summed
term magnitudes; SPAI columns and U-diag factors within 1e-10 / 1e-13; block GMRES
X within 1e-10 of the oracle's replay and every residual <= 1e-8; the coefficient
calls on a problem of roles bit for bit the (s, p) calls; export then import gives
the same preconditioner and the same X bit for bit.
"""
import numpy as np
import pytest
import torch

from synth import config0, gyro_like_job
from oracle.assemble import Assembled
from oracle.diagnostics import fro_I_minus_A, fro_diff
from oracle.spai import SpaiPattern, solve_column
from oracle.update import diag_factors
from oracle.gmres import block_gmres
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx, gpu_P_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


@pytest.fixture(scope="module")
def job():
    return gyro_like_job()


def _problem(ctx, job):
    from paper_1809_06574_amd import Problem
    return Problem(ctx, [(T.rowptr, T.col, T.val) for T in job.aterms])


def test_affine_pattern_maps_and_assembly(ctx, job):
    pb = _problem(ctx, job)
    asm = Assembled(job)
    rp, ci, mp = pb.pattern()
    np.testing.assert_array_equal(np_(rp), asm.rowptr)
    np.testing.assert_array_equal(np_(ci), asm.col)
    for t in range(len(job.aterms)):
        np.testing.assert_array_equal(np_(mp[t]), asm.maps[t])
    for c in job.coefs:
        got = np_(pb.assemble(c))
        want = asm.values_c(c)
        scale = sum(abs(c[t]) * np.abs(asm.values_c(np.eye(len(c))[t])) for t in range(len(c)))
        assert np.all(np.abs(got - want) <= 8 * np.finfo(float).eps * scale)
    # Table 2 norms of the affine points
    v1 = asm.values_c(job.coefs[0])
    for c in job.coefs[1:]:
        a, b = pb.table2_norms_c(job.coefs[0], c)
        vl = asm.values_c(c)
        assert a == pytest.approx(fro_I_minus_A(job.n, asm.rowptr, asm.col, vl), rel=1e-12)
        assert b == pytest.approx(fro_diff(v1, vl), rel=1e-12)


def test_affine_spai_update_and_solve(ctx, job):
    pb = _problem(ctx, job)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    v1 = asm.values_c(job.coefs[0])
    h = pb.spai_build(job.coefs[0], None)
    exp = h.export()
    pv = np_(exp["val"])
    for j in range(0, job.n, 37):
        x, _ = solve_column(job.n, asm.rowptr, asm.col, v1, pat, j)
        got = pv[pat.P_slot[pat.J_colptr[j]:pat.J_colptr[j + 1]]]
        assert np.linalg.norm(got - x) <= 1e-10 * np.linalg.norm(x), j
    B = torch.as_tensor(job.B, device="cuda")
    for l in range(1, len(job.coefs)):
        c = job.coefs[l]
        h.update(c)
        vl = asm.values_c(c)
        q = diag_factors(job.n, asm.rowptr, asm.col, v1, vl)
        np.testing.assert_allclose(np_(h.export()["q"]), q, rtol=1e-13, atol=0)
        X, st, rc = pb.block_solve(h, c, None, B)
        A = to_scipy(job.n, asm.rowptr, asm.col, vl)
        Xg = np_(X)
        rel = np.linalg.norm(job.B - A @ Xg, axis=0) / np.linalg.norm(job.B, axis=0)
        assert np.all(rel <= 1e-8), rel
        Pf = gpu_P_apply(h.export(), job.n)
        Xo, _ = block_gmres(A.__matmul__, Pf, job.B, m=30, tol=1e-8, fixed_steps=st["cycle_steps"])
        assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) <= 1e-10


def test_affine_sequence_batch_and_server_agree(ctx, job):
    """The sequence solve at the affine points equals, bit for bit, a chain of
    coefficient-point updates and solves, a batch of the same items, and the job
    served alone."""
    from paper_1809_06574_amd import batch_solve, Server
    pb = _problem(ctx, job)
    B = torch.as_tensor(job.B, device="cuda")
    X, stats = pb.sequence_solve(B, coefs=job.coefs)
    asm = Assembled(job)
    h = pb.spai_build(job.coefs[0], None)
    for l, c in enumerate(job.coefs):
        if l:
            h.update(c)
        Xl, _, _ = pb.block_solve(h, c, None, B)
        assert torch.equal(Xl, X[l]), l
        vl = asm.values_c(c)
        A = to_scipy(job.n, asm.rowptr, asm.col, vl)
        rel = np.linalg.norm(job.B - A @ np_(X[l]), axis=0) / np.linalg.norm(job.B, axis=0)
        assert np.all(rel <= 1e-8)
    # a batch over the points of one handle: the last point's preconditioner
    Xs, _, sts, rc = batch_solve(ctx, [(pb, h, job.coefs[-1], None, B), (pb, None, job.coefs[1], None, B)])
    assert rc == 0
    assert torch.equal(Xs[0], X[-1])
    X1n, _, _ = pb.block_solve(None, job.coefs[1], None, B)
    assert torch.equal(Xs[1], X1n)
    sv = Server(ctx, k=job.k)
    jid = sv.submit(pb, B, coefs=job.coefs)
    done = []
    while not done:
        done = sv.step()
    (rid, status, Xs_, _), = done
    assert rid == jid and status == 0
    assert torch.equal(Xs_, X)
    sv.close()


def test_role_problem_coefficient_calls_match(ctx):
    """On a problem of roles, the coefficient calls with (s^2, s^2 p, s, s p, 1, p)
    give the (s, p) calls' results bit for bit."""
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    s = job.s
    cf = lambda p: [s * s, s * s * p, s, s * p, 1.0, p]  # noqa: E731
    p0, p2 = job.p_list[0], job.p_list[2]
    assert torch.equal(pb.assemble(s, p2), pb.assemble(cf(p2)))
    h1 = pb.spai_build(s, p0)
    h2 = pb.spai_build(cf(p0), None)
    assert torch.equal(h1.export()["val"], h2.export()["val"])
    h1.update(s, p2)
    h2.update(cf(p2))
    assert torch.equal(h1.export()["q"], h2.export()["q"])
    B = torch.as_tensor(job.B, device="cuda")
    X1, _, _ = pb.block_solve(h1, s, p2, B)
    X2, _, _ = pb.block_solve(h2, cf(p2), None, B)
    assert torch.equal(X1, X2)
    Xa, _ = pb.sequence_solve(B, [s] * 4, job.p_list)
    Xb, _ = pb.sequence_solve(B, coefs=[cf(p) for p in job.p_list])
    assert torch.equal(Xa, Xb)


def test_export_import_round_trip(ctx, job):
    """spai_import of an exported P at the same anchor: the same P, the same X, and
    the same updated preconditioner, bit for bit (problem of roles and affine)."""
    from paper_1809_06574_amd import Problem
    for kind in ("roles", "affine"):
        if kind == "roles":
            j0 = config0()
            pb = Problem(ctx, j0.terms)
            pts = [(j0.s, p) for p in j0.p_list[:3]]
            Bh = j0.B
        else:
            pb = _problem(ctx, job)
            pts = [(c, None) for c in job.coefs[:3]]
            Bh = job.B
        B = torch.as_tensor(Bh, device="cuda")
        h = pb.spai_build(*pts[0])
        e = h.export()
        g = pb.spai_import(pts[0][0], pts[0][1], e["rowptr"], e["col"], e["val"])
        e2 = g.export()
        for key in ("rowptr", "col", "val", "q"):
            assert torch.equal(e[key], e2[key]), (kind, key)
        X1, _, _ = pb.block_solve(h, *pts[0], B)
        X2, _, _ = pb.block_solve(g, *pts[0], B)
        assert torch.equal(X1, X2), kind
        for pt in pts[1:]:
            h.update(*pt)
            g.update(*pt)
            assert torch.equal(h.export()["q"], g.export()["q"]), kind
            X1, _, _ = pb.block_solve(h, *pt, B)
            X2, _, _ = pb.block_solve(g, *pt, B)
            assert torch.equal(X1, X2), kind


def test_affine_argument_errors(ctx, job):
    from paper_1809_06574_amd import lib as L
    import ctypes as C
    pb = _problem(ctx, job)
    # (s, p) calls on an affine problem
    out = torch.empty(pb.nnz, dtype=torch.float64, device="cuda")
    assert L.pmor_assemble(pb.handle, 1.0, 0.5, out.data_ptr()) == L.PMOR_EINVAL
    h = C.c_void_p()
    assert L.spai_build(pb.handle, 1.0, 0.5, None, C.byref(h), None) == L.PMOR_EINVAL
    # a non-finite coefficient
    bad = (C.c_double * 7)(*([1.0] * 6 + [float("nan")]))
    assert L.pmor_assemble_c(pb.handle, bad, out.data_ptr()) == L.PMOR_EINVAL
    # term counts and NULL terms
    T = job.aterms[0]
    rp = torch.as_tensor(T.rowptr, device="cuda")
    ci = torch.as_tensor(T.col, device="cuda")
    va = torch.as_tensor(T.val, device="cuda")
    csr = L.Csr(T.n, T.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    arr = (C.POINTER(L.Csr) * (L.PMOR_TMAX + 1))(*([C.pointer(csr)] * (L.PMOR_TMAX + 1)))
    o = C.c_void_p()
    assert L.pmor_problem_create_affine(ctx.handle, 0, arr, C.byref(o)) == L.PMOR_EINVAL
    assert L.pmor_problem_create_affine(ctx.handle, L.PMOR_TMAX + 1, arr, C.byref(o)) == L.PMOR_EINVAL
    arr2 = (C.POINTER(L.Csr) * 2)(C.pointer(csr), None)
    assert L.pmor_problem_create_affine(ctx.handle, 2, arr2, C.byref(o)) == L.PMOR_EINVAL
    assert L.pmor_problem_create_affine(ctx.handle, L.PMOR_TMAX, arr, C.byref(o)) == L.PMOR_OK
    L.pmor_problem_destroy(o)
    # a malformed imported P (column out of range)
    bad_col = ci.clone()
    bad_col[3] = T.n + 5
    c0 = (C.c_double * 7)(*job.coefs[0])
    assert L.spai_import_c(pb.handle, c0, T.nnz, rp.data_ptr(), bad_col.data_ptr(), va.data_ptr(), None,
                           C.byref(h)) == L.PMOR_EINVAL
