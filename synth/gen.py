"""Seeded generators of parametric second-order systems.

A job is the input of one sequence of solves: sparse terms of
    M(p) = M0 + p*M1,  D(p) = D0 + p*D1,  K(p) = K0 + p*K1
(the second-order system of the paper's eq. (1), each coefficient matrix
affine in one parameter p), a frequency s, a list of parameter values
p_1..p_z and a block of right-hand sides B (n x k).  Absent terms are
simply missing from ``Job.terms``.

Workloads (synthetic stand-ins for the paper's micro-gyroscope model, whose
matrices are a public benchmark not available here):

* ``config0``   2-D 5-point Laplacian 32x32, M = I, D(p) = p*M + 0.01*K, s = 1.
* ``config1``   3-D 7-point grid 64^3 with edge weights U(1,10),
                M = diag U(0.5,1.5), D(p) = p*M + 1e-3*K, s = 2, 20 p in [0.1,1].
* ``config2_system(i)``  one of 512 independent 2-D/3-D systems, n in [4096, 65536],
                with an explicit power-law SPAI pattern (sizes 5..40).
* ``config4_job(j)``  serving jobs, n in {16384, 65536, 262144, 1048576}.
* ``appendix1`` the paper's Appendix I system (non-symmetric, n = 1006).
* ``gyro_like_job``  an affine job with the term structure of the paper's
                micro-gyroscope model (seven matrices, six free coefficients).

Grids are ordered lexicographically with x fastest; Dirichlet boundaries are
modelled by "ghost" edges from each boundary node to the outside, so a
node's diagonal is the sum of all its incident edge weights.  Random draws
use ``numpy.random.default_rng`` with the seeds documented per generator;
the draw order is: edge weights (x-, y-, z-edges, then ghost edges of the
x-, y-, z-faces), then the M diagonal, then p, then B.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

ROLES = ("M0", "M1", "D0", "D1", "K0", "K1")


@dataclasses.dataclass
class CSR:
    """Square sparse matrix in 0-based CSR with sorted, unique column indices."""

    n: int
    rowptr: np.ndarray  # int32, n+1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def scaled(self, alpha: float) -> "CSR":
        return CSR(self.n, self.rowptr.copy(), self.col.copy(), self.val * alpha)


@dataclasses.dataclass
class Job:
    name: str
    n: int
    terms: Dict[str, CSR]
    s: float
    p_list: np.ndarray
    B: np.ndarray  # (n, k) float64, row-major
    pattern: Optional[Tuple[np.ndarray, np.ndarray]] = None  # explicit CSC (colptr, row)
    meta: dict = dataclasses.field(default_factory=dict)
    aterms: Optional[List[CSR]] = None  # affine job: the term matrices T_0..T_{w}
    coefs: Optional[np.ndarray] = None  # affine job: npts x len(aterms) coefficient vectors
    kinds: Optional[List[str]] = None  # complex job: "real", "imag" or "complex" per term

    @property
    def k(self) -> int:
        return int(self.B.shape[1])


def _coo_to_csr(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate entries in generator output")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def _draw_edge_weights(dims, rng, lo, hi):
    """Edge weights of a 2-D (nz == 1) or 3-D grid, in the documented draw order."""
    nx, ny, nz = dims
    three_d = nz > 1
    if rng is None:
        def u(shape):
            return np.full(shape, float(lo))
    else:
        def u(shape):
            return rng.uniform(lo, hi, size=shape)
    wx = u((nz, ny, nx - 1))
    wy = u((nz, ny - 1, nx))
    wz = u((nz - 1, ny, nx)) if three_d else np.zeros((0, ny, nx))
    gx = u((nz, ny, 2))
    gy = u((nz, 2, nx))
    gz = u((2, ny, nx)) if three_d else np.zeros((2, ny, nx))
    return wx, wy, wz, gx, gy, gz


def grid_laplacian(dims, rng=None, lo=1.0, hi=10.0) -> CSR:
    """Weighted graph Laplacian of an nx*ny*nz grid with Dirichlet ghost edges.

    ``rng=None`` gives unit weights (K_ii = 4 in 2-D, 6 in 3-D, K_ij = -1).
    Off-diagonals are -w(edge); the diagonal is the sum of incident weights.
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    wx, wy, wz, gx, gy, gz = _draw_edge_weights(dims, rng, lo, hi)
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    diag = np.zeros((nz, ny, nx))
    rows, cols, vals = [], [], []

    def add_edges(a, b, w):
        a = a.ravel(); b = b.ravel(); w = w.ravel()
        rows.extend([a, b]); cols.extend([b, a]); vals.extend([-w, -w])

    add_edges(idx[:, :, :-1], idx[:, :, 1:], wx)
    diag[:, :, :-1] += wx; diag[:, :, 1:] += wx
    add_edges(idx[:, :-1, :], idx[:, 1:, :], wy)
    diag[:, :-1, :] += wy; diag[:, 1:, :] += wy
    if nz > 1:
        add_edges(idx[:-1], idx[1:], wz)
        diag[:-1] += wz; diag[1:] += wz
    diag[:, :, 0] += gx[:, :, 0]; diag[:, :, -1] += gx[:, :, 1]
    diag[:, 0, :] += gy[:, 0, :]; diag[:, -1, :] += gy[:, 1, :]
    if nz > 1:
        diag[0] += gz[0]; diag[-1] += gz[1]
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def diagonal(values: np.ndarray) -> CSR:
    n = values.size
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.asarray(values, dtype=np.float64).copy())


def config0(k: int = 2) -> Job:
    """2-D 5-point Laplacian 32x32 (n = 1024), M = I, D(p) = p*M + 0.01*K, s = 1.

    p in {0.1, 0.2, 0.3, 0.4}; B = n x 2 of N(0,1), seed 1000.
    """
    dims = (32, 32, 1)
    K = grid_laplacian(dims)
    n = K.n
    M = diagonal(np.ones(n))
    rng = np.random.default_rng(1000)
    B = rng.standard_normal((n, k))
    terms = {"M0": M, "D0": K.scaled(0.01), "D1": M, "K0": K}
    return Job("config0", n, terms, 1.0, np.array([0.1, 0.2, 0.3, 0.4]), B,
               meta={"dims": dims})


def _weighted_mdk(dims, rng, c_damp):
    K = grid_laplacian(dims, rng)
    m = rng.uniform(0.5, 1.5, size=K.n)
    M = diagonal(m)
    return {"M0": M, "D0": K.scaled(c_damp), "D1": M, "K0": K}


def config1(dims=(64, 64, 64), npts: int = 20, k: int = 4, seed: int = 1001) -> Job:
    """3-D 7-point grid (default 64^3, n = 262144), weights U(1,10), M = diag U(0.5,1.5).

    D(p) = p*M + 1e-3*K, s = 2, p_j = linspace(0.1, 1.0, npts), B = n x k N(0,1).
    """
    rng = np.random.default_rng(seed)
    terms = _weighted_mdk(dims, rng, 1e-3)
    n = terms["K0"].n
    p = np.linspace(0.1, 1.0, npts)
    B = rng.standard_normal((n, k))
    return Job("config1", n, terms, 2.0, p, B, meta={"dims": dims})


def _power_law_sizes(rng, n, lo=5, hi=40):
    t = np.arange(lo, hi + 1)
    w = 1.0 / t.astype(np.float64) ** 2
    return rng.choice(t, size=n, p=w / w.sum())


def _nearest_pattern(K: CSR, sizes: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """J_j = the sizes[j] nodes nearest to j by graph distance on K's graph.

    Ties are broken by (distance, index); the set is clamped by availability and
    returned sorted ascending as an explicit CSC pattern (colptr, row).
    """
    n = K.n
    rp, ci = K.rowptr, K.col
    colptr = np.zeros(n + 1, dtype=np.int64)
    rows = []
    for j in range(n):
        want = int(sizes[j])
        chosen = [j]
        frontier = [j]
        seen = {j}
        while len(chosen) < want and frontier:
            nxt = set()
            for u in frontier:
                for e in range(rp[u], rp[u + 1]):
                    v = int(ci[e])
                    if v not in seen:
                        nxt.add(v)
            nxt = sorted(nxt)
            seen.update(nxt)
            take = nxt[: want - len(chosen)]
            chosen.extend(take)
            frontier = nxt
        chosen.sort()
        rows.append(np.array(chosen, dtype=np.int32))
        colptr[j + 1] = colptr[j] + len(chosen)
    return colptr.astype(np.int32), np.concatenate(rows)


def config2_system(i: int, k: int = 8, with_pattern: bool = True) -> Job:
    """System i (0..511) of the batching workload.

    Seed [1002, i].  n_t ~ U{4096..65536}, 2-D or 3-D with probability 1/2;
    2-D: nx = round(sqrt n_t), ny = round(n_t/nx); 3-D: nx = ny = round(n_t^(1/3)),
    nz = round(n_t/nx^2).  M, D, K as config1, s = 2, p ~ U(0.1, 1) and a
    second point p + 0.02.  SPAI pattern sizes follow P(t) ~ t^-2 on [5, 40].
    """
    rng = np.random.default_rng([1002, i])
    n_t = int(rng.integers(4096, 65537))
    three_d = bool(rng.integers(0, 2))
    if three_d:
        nx = ny = int(round(n_t ** (1.0 / 3.0)))
        nz = max(2, int(round(n_t / (nx * nx))))
    else:
        nx = int(round(np.sqrt(n_t)))
        ny = int(round(n_t / nx))
        nz = 1
    dims = (nx, ny, nz)
    terms = _weighted_mdk(dims, rng, 1e-3)
    n = terms["K0"].n
    p0 = float(rng.uniform(0.1, 1.0))
    B = rng.standard_normal((n, k))
    sizes = _power_law_sizes(rng, n)
    pattern = _nearest_pattern(terms["K0"], sizes) if with_pattern else None
    return Job(f"config2_{i}", n, terms, 2.0, np.array([p0, p0 + 0.02]), B, pattern=pattern,
               meta={"dims": dims, "sizes": sizes})


C4_DIMS = ((32, 32, 16), (64, 32, 32), (64, 64, 64), (128, 128, 64))


def config4_job(jid: int, k: int = 4, npts: int = 20, size_class: Optional[int] = None) -> Job:
    """Serving job jid.  Seed [1004, jid].  n uniform over C4_DIMS, p_j = p0 + 0.02 j."""
    rng = np.random.default_rng([1004, jid])
    cls = int(rng.integers(0, len(C4_DIMS))) if size_class is None else int(size_class)
    dims = C4_DIMS[cls]
    terms = _weighted_mdk(dims, rng, 1e-3)
    n = terms["K0"].n
    p0 = float(rng.uniform(0.1, 0.6))
    B = rng.standard_normal((n, k))
    return Job(f"config4_{jid}", n, terms, 2.0, p0 + 0.02 * np.arange(npts), B,
               meta={"dims": dims, "size_class": cls})


def appendix1(s: float = 0.5, p_list=(0.5, 0.6, 0.7, 0.8), k: int = 2, seed: int = 7) -> Job:
    """The system of the paper's Appendix I: A(s,p) = s*I - diag(A1(p), A2, A3, A4).

    A1(p) = [[-1, p], [-p, -1]], A2 = [[-1, 200], [-200, -1]],
    A3 = [[-1, 400], [-400, -1]], A4 = diag(1, ..., 1000); n = 1006.
    Written as D0 = I (coefficient s), K0 = -diag(A1(0), A2, A3, A4) and
    K1 = -[[0, 1], [-1, 0]] in the leading 2x2 block (coefficient p).
    s must avoid {1, ..., 1000} (A4 has positive entries as printed).
    """
    n = 6 + 1000
    r, c, v = [], [], []

    def put(i, j, x):
        r.append(i); c.append(j); v.append(x)

    put(0, 0, 1.0); put(1, 1, 1.0)  # -A1(0) = I in the leading block
    for base, w in ((2, 200.0), (4, 400.0)):
        put(base, base, 1.0); put(base, base + 1, -w)
        put(base + 1, base, w); put(base + 1, base + 1, 1.0)
    for t in range(1000):
        put(6 + t, 6 + t, -float(t + 1))
    K0 = _coo_to_csr(n, np.array(r), np.array(c), np.array(v))
    K1 = _coo_to_csr(n, np.array([0, 1]), np.array([1, 0]), np.array([-1.0, 1.0]))
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, k))
    return Job("appendix1", n, {"D0": diagonal(np.ones(n)), "K0": K0, "K1": K1}, float(s),
               np.asarray(p_list, dtype=np.float64), B)


def tiny_random_job(n: int, density: float, seed: int, k: int = 2, npts: int = 3,
                    roles=("M0", "D0", "D1", "K0"), diag_shift: float = 4.0,
                    symmetric_pattern: bool = False) -> Job:
    """Small non-symmetric random job for brute-force checks.

    Each term gets its own random pattern (density ``density``), so the union
    pattern is a genuine union; K0 also gets ``diag_shift`` on its diagonal so
    that A(s,p) stays safely nonsingular for s, p in [0, 1].
    """
    rng = np.random.default_rng([4242, seed])
    terms = {}
    for role in roles:
        mask = rng.random((n, n)) < density
        if symmetric_pattern:
            mask = mask | mask.T
        vals = rng.standard_normal((n, n))
        if role == "K0":
            mask = mask | np.eye(n, dtype=bool)
            vals = vals + diag_shift * np.eye(n) * np.sqrt(n * density + 1)
        rr, cc = np.nonzero(mask)
        terms[role] = _coo_to_csr(n, rr, cc, vals[rr, cc])
    p = rng.uniform(0.1, 0.9, size=npts)
    B = rng.standard_normal((n, k))
    return Job(f"tiny_{n}_{seed}", n, terms, 0.7, p, B)


def _upwind_x(dims, rng, lo, hi) -> CSR:
    """Non-symmetric first-difference coupling along x: entry (i, i-1) = -w and
    (i, i) = w for every x-edge (weights U(lo, hi)), a convection-like term."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    w = rng.uniform(lo, hi, size=(nz, ny, nx - 1))
    a, b = idx[:, :, 1:].ravel(), idx[:, :, :-1].ravel()
    diag = np.zeros((nz, ny, nx))
    diag[:, :, 1:] += w
    rows = np.concatenate([a, idx.ravel()])
    cols = np.concatenate([b, idx.ravel()])
    vals = np.concatenate([-w.ravel(), diag.ravel()])
    return _coo_to_csr(nx * ny * nz, rows, cols, vals)


def _long_range_x(dims, rng, lo, hi) -> CSR:
    """Symmetric couplings between nodes two apart along x (weights U(lo, hi)),
    Laplacian-like (diagonal = sum of incident weights): a term whose pattern is
    not in the 7-point stencil, so the union pattern is wider than any term."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    w = rng.uniform(lo, hi, size=(nz, ny, nx - 2))
    a, b = idx[:, :, :-2].ravel(), idx[:, :, 2:].ravel()
    diag = np.zeros((nz, ny, nx))
    diag[:, :, :-2] += w
    diag[:, :, 2:] += w
    rows = np.concatenate([a, b, idx.ravel()])
    cols = np.concatenate([b, a, idx.ravel()])
    vals = np.concatenate([-w.ravel(), -w.ravel(), diag.ravel()])
    return _coo_to_csr(nx * ny * nz, rows, cols, vals)


GYRO_POINTS = ((2.0, 0.5, 1.0), (2.0, 0.5, 2.0), (1.5, 0.3, 2.0), (1.5, 0.3, 1.5))


def gyro_coefs(s: float, theta: float, d: float) -> np.ndarray:
    """Coefficients of the seven terms at (s, theta, d), in the order of
    ``gyro_like_job``'s terms: K1 (1), M1 (s^2), M2 (s^2 d), D1 (s theta),
    D2 (s theta d), K2 (1/d), K3 (d) -- the model's free parameters with the
    damping weights alpha = beta = 0."""
    return np.array([1.0, s * s, s * s * d, s * theta, s * theta * d, 1.0 / d, d])


def gyro_like_job(dims=(12, 10, 8), k: int = 2, seed: int = 1010, points=GYRO_POINTS) -> Job:
    """An affine job shaped like the paper's micro-gyroscope model (Section 3):
    s^2 M(d) + s D(theta, d) + K(d) with M(d) = M1 + d M2, D = theta (D1 + d D2),
    K(d) = K1 + (1/d) K2 + d K3, written as seven terms with the coefficients of
    ``gyro_coefs``.  Synthetic stand-ins on a 3-D grid (the model's matrices are
    not available): K1 a weighted Laplacian U(1,10), K2 a weighted Laplacian
    U(0.5,2), K3 couplings two nodes apart U(0.1,0.5), M1 = diag U(0.5,1.5),
    M2 = diag U(0.1,0.3), D1 = 1e-2 times a weighted Laplacian U(1,10), D2 an
    upwind x-difference U(0.5,1) (non-symmetric).  Points: (s, theta, d) in
    ``points`` (the values of d follow the paper's four expansion points; s and
    theta are real here).  Seed ``seed``; draw order K1, K2, K3, M1, M2, D1, D2, B.
    """
    rng = np.random.default_rng(seed)
    K1 = grid_laplacian(dims, rng, 1.0, 10.0)
    K2 = grid_laplacian(dims, rng, 0.5, 2.0)
    K3 = _long_range_x(dims, rng, 0.1, 0.5)
    n = K1.n
    M1 = diagonal(rng.uniform(0.5, 1.5, size=n))
    M2 = diagonal(rng.uniform(0.1, 0.3, size=n))
    D1 = grid_laplacian(dims, rng, 1.0, 10.0).scaled(1e-2)
    D2 = _upwind_x(dims, rng, 0.5, 1.0)
    B = rng.standard_normal((n, k))
    coefs = np.array([gyro_coefs(*pt) for pt in points])
    return Job("gyro_like", n, {}, float("nan"), np.arange(len(points), dtype=np.float64), B,
               meta={"dims": dims, "points": tuple(points),
                     "matrices": {"K1": K1, "M1": M1, "M2": M2, "D1": D1, "D2": D2, "K2": K2, "K3": K3}},
               aterms=[K1, M1, M2, D1, D2, K2, K3], coefs=coefs)


# (f^2, theta, d) of the complex points: s = 2 pi f sqrt(-1), so s^2 = -4 pi^2 f^2
GYRO_COMPLEX_POINTS = ((0.0225, 0.5, 1.0), (0.0225, 0.5, 2.0), (0.02, 0.3, 2.0), (0.015, 0.3, 1.5))
GYRO_KINDS = ("real", "real", "real", "imag", "imag", "real", "real")


def gyro_complex_job(dims=(12, 10, 8), k: int = 2, seed: int = 1010, points=GYRO_COMPLEX_POINTS,
                     rhs_seed: int = 2020) -> Job:
    """The terms of ``gyro_like_job`` at complex points, as in the paper's
    gyroscope example (Section 3): s = 2 pi f sqrt(-1) makes the coefficients of
    M1, M2 (s^2, s^2 d) real and those of D1, D2 (s theta, s theta d) imaginary;
    K1, K2, K3 keep 1, 1/d, d.  The frequencies f^2 in ``points`` follow the
    paper's (0.0225 at two of its four points) and stay below the lowest
    resonance of the synthetic K, M pair; theta is O(1) here so that the
    imaginary part matters.  B is complex: standard normal real and imaginary
    parts, drawn with seed ``rhs_seed`` (real parts first)."""
    base = gyro_like_job(dims, k=1, seed=seed)
    coefs = np.array([gyro_coefs(2j * np.pi * np.sqrt(f2), th, d) for f2, th, d in points])
    rng = np.random.default_rng(rhs_seed)
    B = rng.standard_normal((base.n, k)) + 1j * rng.standard_normal((base.n, k))
    return Job("gyro_complex", base.n, {}, float("nan"), np.arange(len(points), dtype=np.float64), B,
               meta={"dims": dims, "points": tuple(points), "matrices": base.meta["matrices"]},
               aterms=base.aterms, coefs=coefs, kinds=list(GYRO_KINDS))
