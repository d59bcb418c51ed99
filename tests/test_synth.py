"""Seeded input generators: determinism, CSR validity, sizes, and the paper's Appendix I values."""
import hashlib
import os

import numpy as np
import pytest

from synth import config0, config1, config2_system, config4_job, appendix1, grid_laplacian
from oracle.sparse import check_csr, to_dense

HERE = os.path.dirname(os.path.abspath(__file__))


def _digest(job):
    h = hashlib.sha256()
    for role in sorted(job.terms):
        T = job.terms[role]
        for a in (T.rowptr, T.col, T.val):
            h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.ascontiguousarray(job.B).tobytes())
    h.update(np.ascontiguousarray(job.p_list).tobytes())
    return h.hexdigest()


def test_deterministic():
    assert _digest(config0()) == _digest(config0())
    a = config1(dims=(8, 8, 8)); b = config1(dims=(8, 8, 8))
    assert _digest(a) == _digest(b)
    c = config4_job(3); d = config4_job(3)
    assert _digest(c) == _digest(d)


def test_config0_shape():
    j = config0()
    assert j.n == 1024 and j.B.shape == (1024, 2)
    K = j.terms["K0"]
    assert K.nnz == 4992
    check_csr(j.n, K.rowptr, K.col)
    d = K.val[K.col == np.repeat(np.arange(j.n), np.diff(K.rowptr))]
    assert np.all(d == 4.0)
    off = K.val[K.col != np.repeat(np.arange(j.n), np.diff(K.rowptr))]
    assert np.all(off == -1.0)
    np.testing.assert_array_equal(j.p_list, [0.1, 0.2, 0.3, 0.4])


def test_config1_sizes_small_and_full():
    j = config1(dims=(6, 5, 4))
    K = j.terms["K0"]
    check_csr(j.n, K.rowptr, K.col)
    D = to_dense(j.n, K.rowptr, K.col, K.val)
    assert np.allclose(D, D.T)
    # diagonal = sum of incident weights, ghost edges included: equal to the
    # off-diagonal row sum inside the grid, larger by 1..10 per ghost edge on the boundary
    off = D - np.diag(np.diag(D))
    excess = np.diag(D) + off.sum(axis=1)
    nx, ny, nz = 6, 5, 4
    x, y, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    nghost = sum((c == v).astype(int) for c, v in ((x, 0), (x, nx - 1), (y, 0), (y, ny - 1), (z, 0), (z, nz - 1)))
    nghost = nghost.transpose(2, 1, 0).ravel()  # lexicographic, x fastest
    assert np.all(excess[nghost == 0] == pytest.approx(0.0, abs=1e-12))
    assert np.all(excess >= 1.0 * nghost - 1e-12) and np.all(excess <= 10.0 * nghost + 1e-12)
    w = -off[off != 0]
    assert w.min() >= 1.0 and w.max() <= 10.0
    m = j.terms["M0"].val
    assert m.min() >= 0.5 and m.max() <= 1.5
    full = config1()
    assert full.n == 262144 and full.terms["K0"].nnz == 1810432 and full.B.shape == (262144, 4)
    assert full.p_list.size == 20


def test_config2_and_config4_ranges():
    j = config2_system(5, with_pattern=False)
    assert 3000 <= j.n <= 70000 and j.B.shape[1] == 8
    sizes = j.meta["sizes"]
    assert sizes.min() >= 5 and sizes.max() <= 40
    j4 = config4_job(0)
    assert j4.n in (16384, 65536, 262144, 1048576)
    np.testing.assert_allclose(np.diff(j4.p_list), 0.02)


def test_config2_explicit_pattern_small():
    # nearest-neighbour patterns: sorted, contain j, sized min(t_j, reachable)
    from synth.gen import _nearest_pattern, _power_law_sizes
    K = grid_laplacian((7, 6, 1))
    rng = np.random.default_rng(0)
    sizes = _power_law_sizes(rng, K.n)
    cp, rows = _nearest_pattern(K, sizes)
    for jj in range(K.n):
        r = rows[cp[jj]:cp[jj + 1]]
        assert jj in r and np.all(np.diff(r) > 0)
        assert r.size == min(sizes[jj], K.n)


def _read_golden():
    out = {}
    with open(os.path.join(HERE, "golden", "appendix1_blocks.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, r, c, *vals = line.split()
            out[name] = (int(r), int(c), vals)
    return out


def test_appendix1_matches_printed_blocks():
    """The generator's Appendix I system equals the blocks printed in the paper."""
    g = _read_golden()
    for p in (0.0, 0.3, 2.5):
        job = appendix1(s=0.5, p_list=(p,))
        n = job.n
        K = to_dense(n, job.terms["K0"].rowptr, job.terms["K0"].col, job.terms["K0"].val)
        K1 = to_dense(n, job.terms["K1"].rowptr, job.terms["K1"].col, job.terms["K1"].val)
        Kp = K + p * K1  # = -diag(A1(p), A2, A3, A4)
        def block(name):
            r, c, vals = g[name]
            return np.array([[float(v.replace("-p", str(-p)).replace("p", str(p))) for v in vals]]).reshape(r, c)
        np.testing.assert_array_equal(-Kp[0:2, 0:2], block("A1"))
        np.testing.assert_array_equal(-Kp[2:4, 2:4], block("A2"))
        np.testing.assert_array_equal(-Kp[4:6, 4:6], block("A3"))
        tail = -np.diag(Kp)[6:]
        assert tail.size == int(g["A4_size"][2][0])
        assert tail[0] == float(g["A4_first"][2][0]) and tail[-1] == float(g["A4_last"][2][0])
        np.testing.assert_array_equal(tail, np.arange(1, 1001, dtype=float))
        # nothing outside the blocks
        mask = np.zeros((n, n), dtype=bool)
        for b in (0, 2, 4):
            mask[b:b + 2, b:b + 2] = True
        mask[np.arange(6, n), np.arange(6, n)] = True
        assert not np.any(Kp[~mask])
        D0 = job.terms["D0"]
        np.testing.assert_array_equal(to_dense(n, D0.rowptr, D0.col, D0.val), np.eye(n))
