"""Every SpMM variant of the batched engine (1, 2, 4, 8 lanes per row taking a
row's entries in turn; the column split), on the sliced-ELL views and on the
CSR arrays.  The variant is fixed per process, so each runs in a child
process (tests/_spmm_worker.py) on the same systems.

Checks: each variant gives the same X bit for bit from either layout (one
summation order per row); the column split gives the one-lane X bit for bit
(both add a row's entries in order); the autotuner's own choice (no pin) gives
that X bit for bit too, so tuning never changes a result; every X reaches the
1e-8 relative residual against the oracle's assembled A; and all variants
agree to 1e-6.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle.assemble import Assembled
from oracle.sparse import to_scipy

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
VARIANTS = (1, 2, 4, 8, 16, "tuned")


def _run_all(tmp):
    out = {}
    for v in VARIANTS:
        path = os.path.join(tmp, f"x_{v}.npz")
        env = dict(os.environ, PMOR_SPMM_LPR=str(v))
        if v == "tuned":
            env.pop("PMOR_SPMM_LPR")
        env.pop("PMOR_TUNE_CACHE", None)
        print(f"spmm variant {v}", flush=True)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "_spmm_worker.py"), path], env=env,
                           capture_output=True, text=True, timeout=110)
        assert r.returncode == 0, (v, r.stdout[-2000:], r.stderr[-4000:])
        with np.load(path) as z:
            out[v] = {k: z[k] for k in z.files}
    return out


def test_spmm_variants(gpu_lib, tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _spmm_worker import jobs
    res = _run_all(str(tmp_path))
    js = jobs()
    base = res[1]
    for v in VARIANTS:
        got = res[v]
        assert set(got) == set(base)
        for key, X in got.items():
            fmt, i, kind = key.split("_")
            if fmt == "sell":
                assert np.array_equal(X, got[f"csr_{i}_{kind}"]), (v, key)
            if v in (16, "tuned"):
                assert np.array_equal(X, base[key]), (v, key)
            d = np.linalg.norm(X - base[key]) / max(np.linalg.norm(base[key]), 1e-300)
            assert d <= 1e-6, (v, key, d)
    # residuals (the layouts and the one-lane and column-split runs agree bitwise,
    # so one variant of each summation order suffices)
    for v in (1, 2, 4, 8):
        for key, X in res[v].items():
            fmt, i, kind = key.split("_")
            if fmt != "sell":
                continue
            job = js[int(i)]
            p = job.p_list[0] if kind == "p1" else job.p_list[1]
            asm = Assembled(job)
            A = to_scipy(job.n, asm.rowptr, asm.col, asm.values(job.s, p))
            nb = np.linalg.norm(job.B, axis=0)
            rel = np.linalg.norm(job.B - A @ X, axis=0) / np.where(nb > 0, nb, 1.0)
            assert np.all(rel <= 1e-8), (v, key, rel)
