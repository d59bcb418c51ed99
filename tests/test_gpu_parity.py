"""GPU library vs CPU oracle, stage by stage, on the same seeded inputs.

Bars: patterns, index sets and slot maps bit-exact; assembly within a few ulp;
FP64 SPAI / update columns within 1e-10 relative; block GMRES X within 1e-10
relative of the oracle run for the same number of block steps with the GPU's
preconditioner, and every column at relative residual <= 1e-8.
"""
import numpy as np
import pytest
import torch

from synth import config0, tiny_random_job, appendix1, grid_laplacian
from synth.gen import _power_law_sizes, _nearest_pattern, _weighted_mdk, Job
from oracle.assemble import Assembled, term_values_on_pattern
from oracle.spai import SpaiPattern, spai_build, solve_column
from oracle.update import diag_factors, update_diag, update_pattern
from oracle.gmres import block_gmres
from oracle.sparse import to_scipy
from tests._helpers import np_, ctx as make_ctx, col_rel_err, gpu_P_apply

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return make_ctx()


def _jobs():
    return [tiny_random_job(37, 0.1, 1), tiny_random_job(64, 0.06, 2, k=3),
            tiny_random_job(131, 0.03, 3, roles=("M0", "M1", "D0", "D1", "K0", "K1")),
            config0(), appendix1(s=0.5)]


@pytest.mark.parametrize("ji", range(5))
def test_union_pattern_and_maps_bitexact(ctx, ji):
    from paper_1809_06574_amd import Problem
    job = _jobs()[ji]
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    rp, ci, mp = pb.pattern()
    assert pb.nnz == asm.nnz
    np.testing.assert_array_equal(np_(rp), asm.rowptr)
    np.testing.assert_array_equal(np_(ci), asm.col)
    for r, role in enumerate(("M0", "M1", "D0", "D1", "K0", "K1")):
        want = asm.maps.get(role, np.full(asm.nnz, -1, dtype=np.int32))
        np.testing.assert_array_equal(np_(mp[r]), want, err_msg=role)


@pytest.mark.parametrize("ji", range(5))
def test_assembly_values(ctx, ji):
    from paper_1809_06574_amd import Problem
    job = _jobs()[ji]
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    tv = term_values_on_pattern(job.terms, asm.maps, asm.nnz)
    s = job.s
    for p in job.p_list[:2]:
        got = np_(pb.assemble(s, p))
        want = asm.values(s, p)
        # few-ulp agreement relative to the magnitudes of the summed terms
        coef = {"M0": s * s, "M1": s * s * p, "D0": s, "D1": s * p, "K0": 1.0, "K1": p}
        scale = sum(np.abs(coef[r] * tv[r]) for r in coef)
        assert np.all(np.abs(got - want) <= 8 * np.finfo(float).eps * scale)


@pytest.mark.parametrize("ji", range(5))
def test_spai_sets_and_values_f64(ctx, ji):
    from paper_1809_06574_amd import Problem
    job = _jobs()[ji]
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    h = pb.spai_build(job.s, job.p_list[0], stats=True)
    jc, jr, ic, ir = h.export_sets()
    np.testing.assert_array_equal(np_(jc), pat.J_colptr)
    np.testing.assert_array_equal(np_(jr), pat.J_row)
    np.testing.assert_array_equal(np_(ic), pat.I_colptr)
    np.testing.assert_array_equal(np_(ir), pat.I_row)
    exp = h.export()
    np.testing.assert_array_equal(np_(exp["rowptr"]), pat.P_rowptr)
    np.testing.assert_array_equal(np_(exp["col"]), pat.P_col)
    val = asm.values(job.s, job.p_list[0])
    pv, rho = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    err = col_rel_err(job.n, pat.J_colptr, pat.P_slot, np_(exp["val"]), pv)
    assert err <= 1e-10, err
    np.testing.assert_allclose(np_(exp["rho"]), rho, rtol=1e-8, atol=1e-12)
    assert h.last_stats["fro_resid"] == pytest.approx(np.sqrt(np.sum(rho ** 2)), rel=1e-10)


@pytest.mark.parametrize("ji", [0, 3])
def test_spai_values_f32(ctx, ji):
    from paper_1809_06574_amd import Problem
    job = _jobs()[ji]
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    h = pb.spai_build(job.s, job.p_list[0], precision="f32")
    exp = h.export()
    val = asm.values(job.s, job.p_list[0])
    pv, rho = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    err = col_rel_err(job.n, pat.J_colptr, pat.P_slot, np_(exp["val"]), pv)
    assert err <= 1e-4, err
    assert np.all(np_(exp["rho"]) <= (1 + 1e-4) * rho + 1e-5)


@pytest.mark.parametrize("ji", [0, 1, 3])
def test_update_diag_and_pattern(ctx, ji):
    from paper_1809_06574_amd import Problem
    job = _jobs()[ji]
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    v1 = asm.values(job.s, job.p_list[0])
    vl = asm.values(job.s, job.p_list[-1])
    pv1, _ = spai_build(job.n, asm.rowptr, asm.col, v1, pat)
    # U-diag
    h = pb.spai_build(job.s, job.p_list[0], update="diag")
    h.update(job.s, job.p_list[-1])
    exp = h.export()
    q = diag_factors(job.n, asm.rowptr, asm.col, v1, vl)
    np.testing.assert_allclose(np_(exp["q"]), q, rtol=1e-13)
    err = col_rel_err(job.n, pat.J_colptr, pat.P_slot, np_(exp["val"]),
                      update_diag(job.n, pat.P_rowptr, pv1, q))
    assert err <= 1e-10, err
    # same point: q == 1 bit for bit
    h.update(job.s, job.p_list[0])
    assert np.all(np_(h.export()["q"]) == 1.0)
    # U-pattern
    hp = pb.spai_build(job.s, job.p_list[0], update="pattern")
    st = hp.update(job.s, job.p_list[-1], stats=True)
    exq = hp.export()
    qv, rho = update_pattern(job.n, asm.rowptr, asm.col, v1, vl, pat)
    err = col_rel_err(job.n, pat.J_colptr, pat.P_slot, np_(exq["q"]), qv)
    assert err <= 1e-10, err
    assert st["fro_resid"] == pytest.approx(np.sqrt(np.sum(rho ** 2)), rel=1e-9, abs=1e-14)


def _solve_and_check(ctx, job, p_idx=0, k=None, m=30, update=None, precision="f64", tol=1e-8, rebuild=False):
    from paper_1809_06574_amd import Problem
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    h = pb.spai_build(job.s, job.p_list[0], update=update or "diag", precision=precision)
    if p_idx != 0:
        if rebuild:
            h.rebuild(job.s, job.p_list[p_idx])
        else:
            h.update(job.s, job.p_list[p_idx])
    B = job.B if k is None else job.B[:, :k]
    Bd = torch.as_tensor(np.ascontiguousarray(B), device="cuda")
    X, st, rc = pb.block_solve(h, job.s, job.p_list[p_idx], Bd, m=m, tol=tol)
    Xg = np_(X)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[p_idx]))
    # the true residual of the GPU solution, computed on the CPU
    bn = np.linalg.norm(B, axis=0)
    rel = np.linalg.norm(B - A @ Xg, axis=0) / np.where(bn > 0, bn, 1.0)
    assert np.all(rel <= tol * 1.0001), (rel, st)
    # oracle with the GPU's preconditioner, same number of block steps per cycle
    exp = h.export()
    Pf = gpu_P_apply(exp, job.n, update or "diag", q_active=(update == "pattern" and p_idx != 0 and not rebuild))
    Xo, info = block_gmres(A.__matmul__, Pf, B, m=m, tol=tol, fixed_steps=st["cycle_steps"])
    d = np.linalg.norm(Xg - Xo) / max(np.linalg.norm(Xo), 1e-300)
    assert d <= 1e-10, (d, st)
    return st


def test_block_solve_config0_all_points(ctx):
    job = config0()
    for l in range(len(job.p_list)):
        st = _solve_and_check(ctx, job, p_idx=l)
        assert st["cycles"] >= 1 and st["steps"] <= 30


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8, 13, 16])
def test_block_solve_block_sizes(ctx, k):
    job = tiny_random_job(700, 0.006, 50 + k, k=k)
    _solve_and_check(ctx, job, p_idx=1, m=20)


def test_block_solve_pattern_update(ctx):
    job = config0()
    _solve_and_check(ctx, job, p_idx=3, update="pattern")


def test_block_solve_restarts(ctx):
    job = config0()
    st = _solve_and_check(ctx, job, p_idx=0, m=4)
    assert st["cycles"] > 1


def test_appendix1_one_step(ctx):
    """Appendix I: SPAI on pattern(A) is the exact inverse, so one block step; the
    U-diag update of it is not exact any more and takes a second step."""
    job = appendix1(s=0.5)
    st = _solve_and_check(ctx, job, p_idx=2, tol=1e-10, rebuild=True)
    assert st["steps"] == 1
    st = _solve_and_check(ctx, job, p_idx=2, tol=1e-10)
    assert st["steps"] == 2


def test_zero_and_nan_columns(ctx):
    from paper_1809_06574_amd import Problem
    from paper_1809_06574_amd import lib as L
    job = config0(k=3)
    pb = Problem(ctx, job.terms)
    h = pb.spai_build(1.0, 0.1)
    B = np.array(job.B)
    B[:, 1] = 0.0
    X, st, rc = pb.block_solve(h, 1.0, 0.1, torch.as_tensor(B, device="cuda"))
    Xh = np_(X)
    assert np.all(Xh[:, 1] == 0.0) and st["relres"][1] == 0.0
    asm = Assembled(job)
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(1.0, 0.1))
    assert np.linalg.norm(B - A @ Xh) <= 1e-8 * np.linalg.norm(B)
    X0, st0, rc0 = pb.block_solve(h, 1.0, 0.1, torch.zeros((job.n, 2), dtype=torch.float64, device="cuda"))
    assert rc0 == 0 and not np_(X0).any()
    B[5, 0] = np.nan
    _, _, rc = pb.block_solve(h, 1.0, 0.1, torch.as_tensor(B, device="cuda"), raise_on_error=False)
    assert rc == L.PMOR_ENAN


def test_not_converged_reports(ctx):
    from paper_1809_06574_amd import Problem
    from paper_1809_06574_amd import lib as L
    job = config0()
    pb = Problem(ctx, job.terms)
    h = pb.spai_build(1.0, 0.1)
    X, st, rc = pb.block_solve(h, 1.0, 0.1, torch.as_tensor(job.B, device="cuda"), m=2, max_cycles=1,
                               raise_on_error=False)
    assert rc == L.PMOR_ENOTCONV and st["cycles"] == 1 and st["steps"] == 2
    assert all(np.isfinite(st["relres"][:2])) and max(st["relres"][:2]) > 1e-8


def test_singular_column_reported(ctx):
    from paper_1809_06574_amd import Problem
    from paper_1809_06574_amd import lib as L
    job = tiny_random_job(30, 0.15, 9)
    # zero column 7 in every term: A(:, 7) = 0 structurally-present zeros
    terms = {}
    for role, T in job.terms.items():
        v = T.val.copy()
        v[T.col == 7] = 0.0
        terms[role] = (T.rowptr, T.col, v)
    pb = Problem(ctx, terms)
    with pytest.raises(L.PmorError) as e:
        pb.spai_build(job.s, job.p_list[0])
    assert e.value.code == L.PMOR_ESINGULAR


def _explicit_pattern_job(dims, seed):
    rng = np.random.default_rng([777, seed])
    terms = _weighted_mdk(dims, rng, 1e-3)
    K = terms["K0"]
    sizes = _power_law_sizes(rng, K.n)
    sizes[:: max(1, K.n // 7)] = 40  # make sure the large buckets are used
    pat = _nearest_pattern(K, sizes)
    B = rng.standard_normal((K.n, 8))
    return Job(f"explicit_{seed}", K.n, terms, 2.0, np.array([0.3, 0.32]), B, pattern=pat)


@pytest.mark.parametrize("dims,prec", [((17, 13, 1), "f64"), ((7, 6, 5), "f64"), ((9, 8, 7), "f32")])
def test_explicit_power_law_pattern(ctx, dims, prec):
    from paper_1809_06574_amd import Problem
    job = _explicit_pattern_job(dims, dims[0])
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col, explicit=job.pattern)
    h = pb.spai_build(job.s, job.p_list[0], pattern=job.pattern, precision=prec)
    jc, jr, ic, ir = h.export_sets()
    np.testing.assert_array_equal(np_(ic), pat.I_colptr)
    np.testing.assert_array_equal(np_(ir), pat.I_row)
    exp = h.export()
    np.testing.assert_array_equal(np_(exp["rowptr"]), pat.P_rowptr)
    np.testing.assert_array_equal(np_(exp["col"]), pat.P_col)
    val = asm.values(job.s, job.p_list[0])
    pv, rho = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    err = col_rel_err(job.n, pat.J_colptr, pat.P_slot, np_(exp["val"]), pv)
    assert err <= (1e-10 if prec == "f64" else 1e-3), err
    Bd = torch.as_tensor(job.B, device="cuda")
    X, st, rc = pb.block_solve(h, job.s, job.p_list[0], Bd)
    A = to_scipy(job.n, asm.rowptr, asm.col, val)
    rel = np.linalg.norm(job.B - A @ np_(X), axis=0) / np.linalg.norm(job.B, axis=0)
    assert np.all(rel <= 1e-8)


def _dense_block_job():
    """A with a dense 250 x 12 block in its leading columns and an explicit
    pattern whose J_j take three size classes: |J_j| <= 8 (most columns),
    9..64 with short candidate lists, and J_j holding the 12 dense columns,
    whose candidate lists (over 3000 rows before deduplication) exceed the
    LDS sort of the shadow kernels."""
    from synth.gen import _coo_to_csr
    n = 600
    rng = np.random.default_rng([778, 1])
    rr, cc, vv = [], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 8.0), (i + 1, -1.0)):
            if 0 <= j < n:
                rr.append(i); cc.append(j); vv.append(v)
    br, bc = np.meshgrid(np.arange(250), np.arange(12), indexing="ij")
    keep = np.abs(br - bc) > 1
    rr += list(br[keep]); cc += list(bc[keep]); vv += list(0.1 * rng.standard_normal(int(keep.sum())))
    K = _coo_to_csr(n, np.array(rr), np.array(cc), np.array(vv))
    M = _coo_to_csr(n, np.arange(n), np.arange(n), np.ones(n))
    colptr, rows = [0], []
    for j in range(n):
        if j < 20:
            J = set(range(12)) | {j}
        elif 300 <= j < 330:
            J = set(range(j - 6, j + 7))
        else:
            J = {x for x in (j - 1, j, j + 1) if 0 <= x < n}
        rows += sorted(J)
        colptr.append(len(rows))
    pat = (np.array(colptr, dtype=np.int64), np.array(rows, dtype=np.int32))
    B = rng.standard_normal((n, 2))
    return Job("dense_block", n, {"M0": M, "K0": K}, 1.0, np.array([0.5]), B, pattern=pat)


def test_shadow_sets_all_size_classes(ctx):
    from paper_1809_06574_amd import Problem
    job = _dense_block_job()
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col, explicit=job.pattern)
    lens = np.diff(pat.J_colptr)
    assert lens.max() > 8 and lens.min() <= 8
    assert np.diff(pat.I_colptr).max() <= 512
    h = pb.spai_build(job.s, job.p_list[0], pattern=job.pattern)
    jc, jr, ic, ir = h.export_sets()
    np.testing.assert_array_equal(np_(jc), pat.J_colptr)
    np.testing.assert_array_equal(np_(jr), pat.J_row)
    np.testing.assert_array_equal(np_(ic), pat.I_colptr)
    np.testing.assert_array_equal(np_(ir), pat.I_row)
    val = asm.values(job.s, job.p_list[0])
    pv, rho = spai_build(job.n, asm.rowptr, asm.col, val, pat)
    exp = h.export()
    err = col_rel_err(job.n, pat.J_colptr, pat.P_slot, np_(exp["val"]), pv)
    assert err <= 1e-10, err


def test_table2_norms(ctx):
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    for p in job.p_list:
        a, b = pb.table2_norms(1.0, 0.1, 1.0, p)
        assert a == pytest.approx(np.sqrt(1024 * (p + 4.04) ** 2 + 3968 * 1.01 ** 2), rel=1e-12)
        assert b == pytest.approx(abs(p - 0.1) * 32.0, rel=1e-12, abs=1e-14)


def test_sequence_solve_policies(ctx):
    from paper_1809_06574_amd import Problem
    job = config0()
    pb = Problem(ctx, job.terms)
    Bd = torch.as_tensor(job.B, device="cuda")
    asm = Assembled(job)
    for policy in ("update", "rebuild"):
        X, stats = pb.sequence_solve(Bd, [1.0] * 4, job.p_list, policy=policy)
        for l, p in enumerate(job.p_list):
            A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(1.0, p))
            rel = np.linalg.norm(job.B - A @ np_(X[l]), axis=0) / np.linalg.norm(job.B, axis=0)
            assert np.all(rel <= 1e-8), (policy, l, rel)


def test_empty_and_out_of_range_arguments(ctx):
    """Empty and out-of-range inputs: no points, k = 0 or above 16, a leading
    dimension below k, a non-finite s, a preconditioner of another problem are
    rejected with PMOR_EINVAL before any work; an empty batch is a no-op."""
    import ctypes as C
    from paper_1809_06574_amd import Problem
    from paper_1809_06574_amd import lib as L
    job = tiny_random_job(40, 0.1, 3)
    pb = Problem(ctx, job.terms)
    pb2 = Problem(ctx, job.terms)
    h = pb.spai_build(job.s, job.p_list[0])
    B = torch.as_tensor(np.ascontiguousarray(job.B), device="cuda")
    X = torch.zeros_like(B)
    so = L.SolveOpts(30, 20, 1e-8)
    st = L.Stats()

    def solve(hh, s, k, ldb, ldx):
        return L.block_solve(pb.handle, hh, s, 0.5, B.data_ptr(), ldb, k, X.data_ptr(), ldx, C.byref(so),
                             C.byref(st))

    for k in (0, 17, -1):
        assert solve(h.handle, job.s, k, max(k, 1), max(k, 1)) == L.PMOR_EINVAL, k
    assert solve(h.handle, job.s, 2, 1, 2) == L.PMOR_EINVAL
    assert solve(h.handle, float("nan"), 2, 2, 2) == L.PMOR_EINVAL
    assert solve(h.handle, float("inf"), 2, 2, 2) == L.PMOR_EINVAL
    h2 = pb2.spai_build(job.s, job.p_list[0])
    assert solve(h2.handle, job.s, 2, 2, 2) == L.PMOR_EINVAL
    # a sequence of no points
    sl = (C.c_double * 1)(job.s)
    vo = L.SolveOpts(30, 20, 1e-8)
    rc = L.pmor_sequence_solve(pb.handle, B.data_ptr(), 2, 2, sl, sl, 0, X.data_ptr(), 2, L.PMOR_UPDATE, None,
                               C.byref(vo), None)
    assert rc == L.PMOR_EINVAL
    # an empty batch
    assert L.pmor_batch_solve(ctx.handle, None, 0, C.byref(vo), None, None) == L.PMOR_OK
    assert L.pmor_batch_solve(ctx.handle, None, -1, C.byref(vo), None, None) == L.PMOR_EINVAL
    # nothing was written, and the library still solves afterwards
    assert torch.count_nonzero(X).item() == 0
    Xs, sts, rc = pb.block_solve(h, job.s, job.p_list[0], B)
    assert rc == L.PMOR_OK
    for x in (h, h2, pb, pb2):
        x.close()


@pytest.mark.parametrize("which", ["config0", "tiny", "explicit"])
def test_gather_only_block_sums(ctx, which):
    """pmor_spai_gather, the data-movement variant of the least squares: every
    column's block A(I_j, J_j) of the anchor, reduced to its sum, equals the sum of
    the dense block the oracle's index sets pick out (register and LDS buckets)."""
    from paper_1809_06574_amd import Problem
    if which == "config0":
        job, pattern = config0(), None
    elif which == "tiny":
        job, pattern = tiny_random_job(131, 0.03, 3), None
    else:
        job = _explicit_pattern_job((9, 8, 7), 9)
        pattern = job.pattern
    pb = Problem(ctx, job.terms)
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col, explicit=pattern)
    h = pb.spai_build(job.s, job.p_list[0], pattern=pattern)
    got = np_(h.gather_sums())
    A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, job.p_list[0])).toarray()
    for j in range(job.n):
        I = pat.I_row[pat.I_colptr[j]:pat.I_colptr[j + 1]]
        J = pat.J_row[pat.J_colptr[j]:pat.J_colptr[j + 1]]
        blk = A[np.ix_(I, J)]
        assert abs(got[j] - blk.sum()) <= 1e-13 * max(np.abs(blk).sum(), 1e-300), j
