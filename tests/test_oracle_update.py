"""Pins of the oracle's cheap SPAI update (Section 2.3, Table 1; Section 2.4)."""
import numpy as np
import pytest

from synth import config0, tiny_random_job, appendix1
from oracle.assemble import Assembled
from oracle.sparse import to_dense
from oracle.spai import SpaiPattern, spai_build
from oracle.update import diag_factors, update_diag, update_pattern
from oracle.diagnostics import fro_from_residuals


def _setup(job, explicit=None):
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col, explicit=explicit)
    return asm, pat


def _dense(n, pat, v):
    return to_dense(n, pat.P_rowptr, pat.P_col, v)


def test_same_point_gives_identity_bitwise():
    """(i) p_l = p_1: q = 1 exactly, so P_l = P_1 bit for bit."""
    job = tiny_random_job(21, 0.15, 1)
    asm, pat = _setup(job)
    v1 = asm.values(job.s, job.p_list[0])
    pv1, _ = spai_build(job.n, asm.rowptr, asm.col, v1, pat)
    q = diag_factors(job.n, asm.rowptr, asm.col, v1, v1.copy())
    assert np.all(q == 1.0)
    np.testing.assert_array_equal(update_diag(job.n, pat.P_rowptr, pv1, q), pv1)


def test_full_patterns_give_exact_inverse():
    """(ii) full Q and P_1 patterns: Q_l P_1 = A(l)^{-1}."""
    job = tiny_random_job(18, 0.2, 2)
    n = job.n
    full = (np.arange(n + 1, dtype=np.int32) * n, np.tile(np.arange(n, dtype=np.int32), n))
    asm, pat = _setup(job, explicit=full)
    v1 = asm.values(job.s, job.p_list[0]); vl = asm.values(job.s, job.p_list[2])
    pv1, _ = spai_build(n, asm.rowptr, asm.col, v1, pat)
    qv, rho = update_pattern(n, asm.rowptr, asm.col, v1, vl, pat)
    Pl = _dense(n, pat, qv) @ _dense(n, pat, pv1)
    Al = to_dense(n, asm.rowptr, asm.col, vl)
    kappa = np.linalg.cond(Al)
    np.testing.assert_allclose(Pl, np.linalg.inv(Al), atol=1e-12 * kappa * np.abs(np.linalg.inv(Al)).max())
    assert fro_from_residuals(rho) <= 1e-12 * kappa * np.linalg.norm(to_dense(n, asm.rowptr, asm.col, v1))


@pytest.mark.parametrize("seed", range(3))
def test_update_two_sided_bound(seed):
    """(iii) rebuilt <= updated <= ||I - A(1)P_1|| + ||A(1) - A(l)Q||_F ||P_1||_2 (U-diag)."""
    job = tiny_random_job(26, 0.15, 20 + seed, npts=4)
    n = job.n
    asm, pat = _setup(job)
    v1 = asm.values(job.s, job.p_list[0])
    pv1, rho1 = spai_build(n, asm.rowptr, asm.col, v1, pat)
    P1 = _dense(n, pat, pv1)
    A1 = to_dense(n, asm.rowptr, asm.col, v1)
    for p in job.p_list[1:]:
        vl = asm.values(job.s, p)
        Al = to_dense(n, asm.rowptr, asm.col, vl)
        q = diag_factors(n, asm.rowptr, asm.col, v1, vl)
        Pupd = _dense(n, pat, update_diag(n, pat.P_rowptr, pv1, q))
        pvr, _ = spai_build(n, asm.rowptr, asm.col, vl, pat)
        Preb = _dense(n, pat, pvr)
        upd = np.linalg.norm(np.eye(n) - Al @ Pupd)
        reb = np.linalg.norm(np.eye(n) - Al @ Preb)
        bound = (np.linalg.norm(np.eye(n) - A1 @ P1)
                 + np.linalg.norm(A1 - Al @ np.diag(q)) * np.linalg.norm(P1, 2))
        assert reb <= upd * (1 + 1e-12)
        assert upd <= bound * (1 + 1e-12)


def test_diag_factor_is_one_column_lstsq():
    """(v) each q_i equals the SVD least-squares solution of min ||A(1)e_i - q A(l)e_i||."""
    job = tiny_random_job(23, 0.2, 5)
    n = job.n
    asm, _ = _setup(job)
    v1 = asm.values(job.s, job.p_list[0]); vl = asm.values(job.s, job.p_list[1])
    q = diag_factors(n, asm.rowptr, asm.col, v1, vl)
    A1 = to_dense(n, asm.rowptr, asm.col, v1); Al = to_dense(n, asm.rowptr, asm.col, vl)
    for i in range(n):
        x, *_ = np.linalg.lstsq(Al[:, [i]], A1[:, i], rcond=None)
        assert q[i] == pytest.approx(x[0], rel=1e-13)


def test_pattern_update_columns_match_full_lstsq():
    job = tiny_random_job(22, 0.15, 6)
    n = job.n
    asm, pat = _setup(job)
    v1 = asm.values(job.s, job.p_list[0]); vl = asm.values(job.s, job.p_list[1])
    qv, rho = update_pattern(n, asm.rowptr, asm.col, v1, vl, pat)
    A1 = to_dense(n, asm.rowptr, asm.col, v1); Al = to_dense(n, asm.rowptr, asm.col, vl)
    Q = _dense(n, pat, qv)
    for i in range(n):
        J = pat.J(i)
        x, *_ = np.linalg.lstsq(Al[:, J], A1[:, i], rcond=None)
        np.testing.assert_allclose(Q[J, i], x, rtol=1e-11, atol=1e-13)
    # ||A(1) - A(l) Q||_F from the column residuals (Section 2.4, the last display)
    assert np.linalg.norm(A1 - Al @ Q) == pytest.approx(fro_from_residuals(rho), rel=1e-10)


def test_appendix1_pattern_update_is_identity_outside_leading_block():
    """(iv) Appendix I: A(l) - A(1) lives in the leading 2x2 block, so Q e_i = e_i for i >= 2."""
    job = appendix1(s=0.5)
    n = job.n
    asm, pat = _setup(job)
    v1 = asm.values(0.5, job.p_list[0])
    for p in job.p_list[1:]:
        vl = asm.values(0.5, p)
        cols = list(range(0, 12)) + [500, 1005]
        qv, rho = update_pattern(n, asm.rowptr, asm.col, v1, vl, pat, columns=cols)
        Q = _dense(n, pat, np.nan_to_num(qv))
        for i in cols[2:]:
            e = np.zeros(n); e[i] = 1.0
            np.testing.assert_allclose(Q[:, i], e, atol=1e-14)
            assert rho[i] <= 1e-13
        # the leading block is the exact 2x2 solve A1(l)^{-1} A1(1)
        Al = to_dense(n, asm.rowptr, asm.col, vl)[:2, :2]
        A1 = to_dense(n, asm.rowptr, asm.col, v1)[:2, :2]
        np.testing.assert_allclose(Q[:2, :2], np.linalg.solve(Al, A1), rtol=1e-13)


def test_config0_update_quality_ratio():
    """C0: the U-diag update stays within the two-sided bound along the whole sequence."""
    job = config0()
    n = job.n
    asm, pat = _setup(job)
    v1 = asm.values(1.0, job.p_list[0])
    pv1, rho1 = spai_build(n, asm.rowptr, asm.col, v1, pat)
    for p in job.p_list[1:]:
        vl = asm.values(1.0, p)
        q = diag_factors(n, asm.rowptr, asm.col, v1, vl)
        # M = I and D1 = M, so A(l) = A(1) + dp I: q_i has the closed form
        # (a_i . a_i + dp a_ii) / (a_i . a_i + 2 dp a_ii + dp^2), a_i = A(1) e_i
        A1 = to_dense(n, asm.rowptr, asm.col, v1)
        dp = p - job.p_list[0]
        nn = np.sum(A1 * A1, axis=0); dd = np.diag(A1)
        np.testing.assert_allclose(q, (nn + dp * dd) / (nn + 2 * dp * dd + dp * dp), rtol=1e-14)


# ---- second approach (Table 1, right column: anchor A(l-1), P_l = Q_l P_{l-1}) ----

def test_second_approach_first_step_is_the_first_approach():
    """At l = 2 both approaches anchor at A(1): the same P_2 bit for bit."""
    from oracle.update import second_approach_diag
    job = tiny_random_job(23, 0.15, 41, npts=4)
    asm, pat = _setup(job)
    vals = [asm.values(job.s, p) for p in job.p_list]
    pv1, _ = spai_build(job.n, asm.rowptr, asm.col, vals[0], pat)
    Ps, qs = second_approach_diag(job.n, asm.rowptr, asm.col, vals, pat.P_rowptr, pv1)
    q_first = diag_factors(job.n, asm.rowptr, asm.col, vals[0], vals[1])
    np.testing.assert_array_equal(qs[1], q_first)
    np.testing.assert_array_equal(Ps[1], update_diag(job.n, pat.P_rowptr, pv1, q_first))
    # later points differ from the first approach (the anchors differ)
    q3_first = diag_factors(job.n, asm.rowptr, asm.col, vals[0], vals[2])
    assert not np.allclose(Ps[2], update_diag(job.n, pat.P_rowptr, pv1, q3_first), rtol=1e-12, atol=0)


def test_second_approach_diagonal_matrices_telescope_to_the_inverse():
    """Diagonal A(l) = diag(d_l): P_1 = diag(1/d_1), the step factors are
    q_l = d_{l-1} / d_l, and their product telescopes, so P_L = diag(1/d_L) =
    A(L)^{-1} (as the first approach gives it)."""
    from oracle.update import second_approach_diag
    n, L = 40, 7
    rng = np.random.default_rng(5)
    d = [rng.uniform(0.5, 3.0, n) * rng.choice([-1.0, 1.0], n) for _ in range(L)]
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    Ps, qs = second_approach_diag(n, rowptr, col, d, rowptr, 1.0 / d[0])
    for l in range(1, L):
        np.testing.assert_allclose(qs[l], d[l - 1] / d[l], rtol=1e-15)
        np.testing.assert_allclose(Ps[l], 1.0 / d[l], rtol=4e-15 * l)
        q_first = diag_factors(n, rowptr, col, d[0], d[l])
        np.testing.assert_allclose(Ps[l], update_diag(n, rowptr, 1.0 / d[0], q_first), rtol=4e-15 * l)


def test_second_approach_dense_brute_force():
    """Each step as a dense one-unknown least squares per column
    (numpy.linalg.lstsq on A(l)(:, i) against A(l-1)(:, i)), the products
    diag(q_l) P_{l-1} formed densely."""
    from oracle.update import second_approach_diag
    job = tiny_random_job(16, 0.2, 43, npts=5)
    n = job.n
    asm, pat = _setup(job)
    vals = [asm.values(job.s, p) for p in job.p_list]
    pv1, _ = spai_build(n, asm.rowptr, asm.col, vals[0], pat)
    Ps, _ = second_approach_diag(n, asm.rowptr, asm.col, vals, pat.P_rowptr, pv1)
    P = _dense(n, pat, pv1)
    for l in range(1, len(vals)):
        Aprev = to_dense(n, asm.rowptr, asm.col, vals[l - 1])
        Al = to_dense(n, asm.rowptr, asm.col, vals[l])
        q = np.array([np.linalg.lstsq(Al[:, [i]], Aprev[:, i], rcond=None)[0][0] for i in range(n)])
        P = np.diag(q) @ P
        np.testing.assert_allclose(_dense(n, pat, Ps[l]), P, rtol=1e-13, atol=1e-15 * np.abs(P).max())


# ---- re-anchoring (rebuild P where the first-approach update misfits) ----

def test_misfit_is_the_dense_frobenius_ratio():
    from oracle.update import misfit_diag
    job = tiny_random_job(19, 0.2, 44, npts=3)
    n = job.n
    asm, _ = _setup(job)
    va, vl = asm.values(job.s, job.p_list[0]), asm.values(job.s, job.p_list[2])
    q = diag_factors(n, asm.rowptr, asm.col, va, vl)
    Aa, Al = to_dense(n, asm.rowptr, asm.col, va), to_dense(n, asm.rowptr, asm.col, vl)
    want = np.linalg.norm(Aa - Al @ np.diag(q), "fro") / np.linalg.norm(Aa, "fro")
    assert misfit_diag(n, asm.rowptr, asm.col, va, vl) == pytest.approx(want, rel=1e-12)
    assert misfit_diag(n, asm.rowptr, asm.col, va, va.copy()) == 0.0


def test_plan_anchors_limits_and_a_jump():
    from oracle.update import misfit_diag, plan_anchors
    job = tiny_random_job(30, 0.15, 45)
    n = job.n
    asm, _ = _setup(job)
    ps = [0.1, 0.11, 0.12, 3.0, 3.01, 3.02]
    vals = [asm.values(job.s, p) for p in ps]
    assert plan_anchors(n, asm.rowptr, asm.col, vals, np.inf) == [0]
    assert plan_anchors(n, asm.rowptr, asm.col, vals, 0.0) == list(range(len(ps)))
    small = max(misfit_diag(n, asm.rowptr, asm.col, vals[a], vals[b]) for a, b in ((0, 1), (0, 2), (3, 4), (3, 5)))
    big = misfit_diag(n, asm.rowptr, asm.col, vals[0], vals[3])
    assert big > 10 * small
    assert plan_anchors(n, asm.rowptr, asm.col, vals, np.sqrt(small * big)) == [0, 3]


# ---- adaptive Q pattern (diagonal, escalated to J_i where the diagonal misfits) ----

def test_adaptive_limits_and_monotone_misfit():
    """ep = inf keeps every column diagonal (Q = diag(q)); ep = 0 escalates
    every column with a nonzero misfit (Q = the U-pattern Q); in between each
    column is one of the two, and the escalated columns' residuals are at most
    their diagonal misfit (J_i holds i, so the diagonal is a candidate of the
    pattern least squares)."""
    from oracle.update import update_adaptive
    job = tiny_random_job(24, 0.15, 46, npts=3)
    n = job.n
    asm, pat = _setup(job)
    v1, vl = asm.values(job.s, job.p_list[0]), asm.values(job.s, job.p_list[2])
    q = diag_factors(n, asm.rowptr, asm.col, v1, vl)
    qd, rd, esc = update_adaptive(n, asm.rowptr, asm.col, v1, vl, pat, np.inf)
    assert esc == []
    np.testing.assert_array_equal(_dense(n, pat, qd), np.diag(q))
    qp, rp = update_pattern(n, asm.rowptr, asm.col, v1, vl, pat)
    qa, ra, esc0 = update_adaptive(n, asm.rowptr, asm.col, v1, vl, pat, 0.0)
    assert esc0 == [i for i in range(n) if rd[i] > 0] and len(esc0) >= n - 2
    for i in esc0:
        a, b = pat.J_colptr[i], pat.J_colptr[i + 1]
        np.testing.assert_array_equal(qa[pat.P_slot[a:b]], qp[pat.P_slot[a:b]])
        assert ra[i] == rp[i]
    assert np.all(rp <= rd * (1 + 1e-12) + 1e-15)
    ratios = rd / np.array([np.linalg.norm(to_dense(n, asm.rowptr, asm.col, v1)[:, i]) for i in range(n)])
    ep = float(np.median(ratios))
    qm, rm, escm = update_adaptive(n, asm.rowptr, asm.col, v1, vl, pat, ep)
    assert 0 < len(escm) < n and set(escm) == set(np.nonzero(ratios > ep)[0].tolist())
    for i in range(n):
        a, b = pat.J_colptr[i], pat.J_colptr[i + 1]
        src = qp if i in escm else qd
        np.testing.assert_array_equal(qm[pat.P_slot[a:b]], src[pat.P_slot[a:b]])
    assert np.sqrt(np.sum(rp ** 2)) <= np.sqrt(np.sum(rm ** 2)) <= np.sqrt(np.sum(rd ** 2))
