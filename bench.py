#!/usr/bin/env python3
"""Parametric solves per second at relative residual 1e-8: SPAI update vs rebuild.

A step is one job of the sequence of Section 2.3 (eq. general_sq) on the
3-D 7-point workload (64^3 grid, n = 262144, k = 4 right-hand sides, s = 2,
20 points p_j in [0.1, 1]): pattern setup of A(s,p) = s^2 M + s D(p) + K,
SPAI P_1 of A(p_1), the cheap first-approach update P_j = diag(q) P_1 of every
later point, and block GMRES(30) for all 20 systems, every column to relative
residual <= 1e-8.  The points only depend on P_1, so the library solves them
together (one launch per kernel per block step for all unfinished points).
Inputs (term matrices, B) are resident on the GPU before the timed region.
`value` = solves/s of that policy over the timed steps.  Beside it: the rebuild
policy (a fresh SPAI per point) solved the same way, both policies point after
point, and the plain path (one right-hand side per solve, a rebuild per
point); per-solve latency = job submission to the point's final X (p50/p99).

The dominant kernel is timed with HIP events on the library's stream during
the timed region (library kernel timer), giving the roofline object; the CPU
oracle is timed on a bounded sample of the same job (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def run_job(pb_factory, job, B, policy, mode="batched", lat=None, Xbuf=None, approach="first", steps=None,
            update="diag", adapt_ep=0.0):
    """One job; returns the number of parametric solves.  lat collects, per point,
    the seconds from the job's submission until the point's X is final.

    batched:   pmor_sequence_solve: P_1, then every point's update (or rebuild)
               and all points' block GMRES solved together;
    pointwise: point after point, spai_update/spai_rebuild then block_solve;
    plain:     point after point, spai_rebuild then one non-block GMRES per column.
    approach:  the update's anchor (Table 1): "first" A(1), "second" A(l-1);
    update:    the pattern of Q ("diag", "pattern", "adaptive" with adapt_ep).
    steps collects the block steps of every point (batched mode).
    """
    s = job.s
    npts = len(job.p_list)
    t_job = time.perf_counter()
    pb = pb_factory()
    if mode == "batched":
        t_call = time.perf_counter()
        _, stats = pb.sequence_solve(B, [s] * npts, job.p_list, policy=policy, X=Xbuf, approach=approach,
                                     update=update, adapt_ep=adapt_ep)
        if steps is not None:
            steps += [sum(st["cycle_steps"]) for st in stats]
        if lat is not None:
            lat += [(t_call - t_job) + st["t_solve_ms"] * 1e-3 for st in stats]
        pb.close()
        return npts
    h = pb.spai_build(s, job.p_list[0])
    for l, p in enumerate(job.p_list):
        if l > 0:
            if policy == "update":
                h.update(s, p)
            else:
                h.rebuild(s, p)
        if mode == "plain":
            for c in range(B.shape[1]):
                pb.block_solve(h, s, p, B[:, c:c + 1].contiguous())
        else:
            pb.block_solve(h, s, p, B, X=Xbuf[l] if Xbuf is not None else None)
        if lat is not None:
            lat.append(time.perf_counter() - t_job)
    h.close()
    pb.close()
    return npts


def timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    for _ in range(steps):
        n += fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, n


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_spai_cols(args):
    """Pool worker: the oracle's SPAI columns `cols` of the C1 job (fresh process)."""
    cols, = args
    from synth import config1
    from oracle.assemble import Assembled
    from oracle.spai import SpaiPattern, spai_build
    job = config1()
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    v1 = asm.values(job.s, job.p_list[0])
    t = time.perf_counter()
    pv, _ = spai_build(job.n, asm.rowptr, asm.col, v1, pat, columns=cols)
    idx = np.concatenate([pat.P_slot[pat.J_colptr[j]:pat.J_colptr[j + 1]] for j in cols])
    return idx, pv[idx], time.perf_counter() - t


def cpu_baseline(job, kept=None):
    """The oracle on the C1 job, two ways, on the machine's host cores:
    (i)  one process, NumPy/SciPy with BLAS threads = the cores: the pattern
         setup, the SPAI of a strided 1/8 of the columns (scaled to all), and the
         U-diag update and block GMRES(30) solve at the first, middle and last
         point (mean over the job's points);
    (ii) the SPAI columns split over a pool of one process per core (all
         columns, measured), then the same update and solves, with the oracle's
         own P_1 from the pool (run (i) uses it too).
    kept: {precision: {point: X}} from the GPU runs; each is compared with the
    oracle's FP64 solution at that point (block GMRES(30) to 1e-12 with the
    oracle's P_1)."""
    import multiprocessing as mp
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = None
    from oracle.assemble import Assembled
    from oracle.spai import SpaiPattern, spai_build
    from oracle.update import diag_factors, update_diag
    from oracle.sparse import to_scipy
    from oracle.gmres import block_gmres
    ncores = min(16, os.cpu_count() or 1)
    t = time.perf_counter()
    asm = Assembled(job)
    pat = SpaiPattern(job.n, asm.rowptr, asm.col)
    t_setup = time.perf_counter() - t
    v1 = asm.values(job.s, job.p_list[0])
    # (ii) the full SPAI over a pool of processes
    _note("cpu baseline: SPAI columns over a process pool")
    chunks = [np.arange(c, job.n, ncores) for c in range(ncores)]
    P1 = np.zeros(pat.J_row.size)
    pool = mp.get_context("spawn").Pool(ncores)
    try:
        t = time.perf_counter()
        for idx, vals, _ in pool.imap_unordered(_oracle_spai_cols, [(c,) for c in chunks]):
            P1[idx] = vals
        t_build_pool = time.perf_counter() - t
    finally:
        pool.close()
        pool.join()
    # (i) one process: a strided eighth of the columns, scaled
    _note("cpu baseline: SPAI sample in one process")
    cols = np.arange(0, job.n, 8)
    t = time.perf_counter()
    spai_build(job.n, asm.rowptr, asm.col, v1, pat, columns=cols)
    t_build_one = (time.perf_counter() - t) * job.n / len(cols)
    npts = len(job.p_list)
    t_upd, t_solve, steps = [], [], []
    for l in (0, npts // 2, npts - 1):
        _note(f"cpu baseline: point {l}")
        vl = asm.values(job.s, job.p_list[l])
        t = time.perf_counter()
        q = diag_factors(job.n, asm.rowptr, asm.col, v1, vl)
        Pl = update_diag(job.n, pat.P_rowptr, P1, q)
        t_upd.append(time.perf_counter() - t)
        A = to_scipy(job.n, asm.rowptr, asm.col, vl)
        P = to_scipy(job.n, pat.P_rowptr, pat.P_col, Pl)
        t = time.perf_counter()
        _, info = block_gmres(A.__matmul__, P.__matmul__, job.B, m=30, tol=1e-8)
        t_solve.append(time.perf_counter() - t)
        steps.append(sum(info.steps))
    vs_oracle = {}
    if kept:
        _note("cpu baseline: FP64 oracle solutions for the precision comparison")
        pts = sorted(next(iter(kept.values())).keys())
        for l in pts:
            vl = asm.values(job.s, job.p_list[l])
            q = diag_factors(job.n, asm.rowptr, asm.col, v1, vl)
            A = to_scipy(job.n, asm.rowptr, asm.col, vl)
            P = to_scipy(job.n, pat.P_rowptr, pat.P_col, update_diag(job.n, pat.P_rowptr, P1, q))
            Xo, _ = block_gmres(A.__matmul__, P.__matmul__, job.B, m=30, tol=1e-12, max_cycles=40)
            for prec, xs in kept.items():
                d = float(np.linalg.norm(xs[l] - Xo) / np.linalg.norm(Xo))
                vs_oracle.setdefault(prec, {})[str(l)] = d
    per_points = (npts - 1) * float(np.mean(t_upd)) + npts * float(np.mean(t_solve))
    job_one = t_setup + t_build_one + per_points
    job_pool = t_setup + t_build_pool + per_points
    return {"value": npts / job_pool, "unit": "solves/s", "cores": ncores, "kind": "oracle",
            "sample": (f"one {job.name} job: pattern setup {t_setup:.2f}s; SPAI of all {job.n} columns over a "
                       f"pool of {ncores} processes {t_build_pool:.1f}s (measured); U-diag update "
                       f"{np.mean(t_upd):.2f}s and block GMRES(30) solve {np.mean(t_solve):.2f}s with the oracle's "
                       f"own P_1 (mean of points 0, {npts // 2}, {npts - 1}, steps {steps}, scaled to {npts} "
                       f"points); update policy"),
            "single_process": {"value": npts / job_one, "unit": "solves/s", "blas_threads": blas_threads,
                               "spai_s": t_build_one,
                               "sample": f"SPAI of {len(cols)} of {job.n} columns in one process, scaled"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "precision_rel_err_vs_oracle_f64": vs_oracle}


def _scrub(dev, gib=1):
    """Write a 1 GiB buffer so that no operand of the next call sits in L2 or the memory-side cache."""
    import torch
    buf = torch.empty((gib << 27,), dtype=torch.float64, device=dev)
    buf.fill_(1.0)
    torch.cuda.synchronize()
    del buf


def spmm_rooflines(ctx, L, sizes=((64, 64, 64, 20), (128, 128, 64, 20), (128, 128, 256, 4))):
    """The engine's SpMM with A and with the preconditioner inside the sequence
    solve (U-diag update, all points together), after a 1 GiB scrub, at C1, C4's
    largest class and a 128 x 128 x 256 stand-in: GB/s in distinct bytes (A's
    pattern and P_1 once per launch), from the library's HIP-event timer."""
    import torch
    from synth import config1
    from paper_1809_06574_amd import Problem
    out = {}
    for nx, ny, nz, npts in sizes:
        _note(f"spmm rooflines: {nx}x{ny}x{nz}, {npts} points")
        job = config1(dims=(nx, ny, nz), npts=npts, k=4, seed=1001)
        dev = ctx.device
        terms = {r: (torch.as_tensor(T.rowptr, device=dev), torch.as_tensor(T.col, device=dev),
                     torch.as_tensor(T.val, device=dev)) for r, T in job.terms.items()}
        B = torch.as_tensor(job.B, device=dev)
        X = torch.empty((npts,) + tuple(B.shape), dtype=torch.float64, device=dev)
        pb = Problem(ctx, terms)
        pb.sequence_solve(B, [job.s] * npts, job.p_list, X=X)  # untimed: buffers, tuning
        rec = {"n": job.n, "nnz": pb.nnz, "points": npts}
        for name in ("spmm_a", "spmm_p"):
            _scrub(dev)
            L.check(L.pmor_prof_set(ctx.handle, L.PROF_KERNELS[name]), "prof_set")
            pb.sequence_solve(B, [job.s] * npts, job.p_list, X=X)
            n_, ms_, by_ = _prof_read(L, ctx)
            L.check(L.pmor_prof_set(ctx.handle, 0), "prof_set")
            rec[name] = {"launches": n_, "avg_us": 1e3 * ms_ / max(n_, 1), "GBps": by_ / max(ms_ * 1e-3, 1e-12) / 1e9,
                         "bytes_per_launch": by_ / max(n_, 1)}
            rec[name]["frac"] = rec[name]["GBps"] / HBM_PEAK_GBS
            # the streaming ceiling at the launch's mix of distinct bytes: blocks of
            # n kp doubles per point, W written (A) or V_j and Z written (P)
            blk = 8.0 * job.n * 4 * npts
            wr = 1 if name == "spmm_a" else 2
            at, rates = mix_ceiling(ctx, L, blk, rec[name]["bytes_per_launch"] / blk - wr, wr, {})
            rec[name]["stream_ceiling"] = {"reads_blocks": rec[name]["bytes_per_launch"] / blk - wr,
                                           "writes_blocks": wr, "at_mix_GBps": at, "rates": rates}
            rec[name]["frac_of_stream_ceiling"] = rec[name]["GBps"] / at
        pb.close()
        del terms, B, X
        torch.cuda.synchronize()
        out[f"{nx}x{ny}x{nz}"] = rec
    return out


def spai_rooflines(ctx, L, factory, job):
    """The SPAI of the C1 job after a 1 GiB scrub: the gather-only variant
    (pmor_spai_gather) against HBM (algorithmic bytes: A once, the index sets, the
    sums), and the FP64 least squares in GFLOP/s (2 |J|^2 (|I| - |J|/3) per column)."""
    import torch
    pb = factory()
    h = pb.spai_build(job.s, job.p_list[0])
    h.gather_sums()  # untimed
    _scrub(ctx.device)
    L.check(L.pmor_prof_set(ctx.handle, L.PROF_SPAI_GATHER), "prof_set")
    h.gather_sums()
    n_, ms_, by_ = _prof_read(L, ctx)
    gather = {"launches": n_, "ms": ms_, "GBps": by_ / max(ms_ * 1e-3, 1e-12) / 1e9, "bytes": by_}
    gather["frac"] = gather["GBps"] / HBM_PEAK_GBS
    _scrub(ctx.device)
    L.check(L.pmor_prof_set(ctx.handle, L.PROF_KERNELS["spai_ls"]), "prof_set")
    h.rebuild(job.s, job.p_list[0])
    n2, ms2, by2 = _prof_read(L, ctx)
    L.check(L.pmor_prof_set(ctx.handle, 0), "prof_set")
    jc, _, ic, _ = h.export_sets()
    nj = torch.diff(jc.to(torch.float64))
    ni = torch.diff(ic.to(torch.float64))
    flops = float(torch.sum(2.0 * nj * nj * (ni - nj / 3.0)))
    h.close()
    pb.close()
    return {"gather_only": gather,
            "least_squares_f64": {"ms": ms2, "gflop": flops / 1e9, "GFLOPs": flops / max(ms2 * 1e-3, 1e-12) / 1e9,
                                  "GBps": by2 / max(ms2 * 1e-3, 1e-12) / 1e9}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config1", choices=["config1", "config0"])
    ap.add_argument("--roofline-kernel", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-arms", action="store_true", help="time only the update policy")
    ap.add_argument("--serve-jobs", type=int, default=200, help="jobs per serving run (0: no serving run)")
    ap.add_argument("--c2-systems", type=int, default=512, help="systems of the batch run (0: none)")
    ap.add_argument("--no-precisions", action="store_true", help="skip the least-squares precision runs")
    ap.add_argument("--no-rooflines", action="store_true", help="skip the SpMM / gather / least-squares rooflines")
    ap.add_argument("--spmm-sizes", default="64x64x64x20,128x128x64x20,128x128x256x4",
                    help="grids and point counts of the SpMM rooflines (nx x ny x nz x points, comma-separated; "
                         "'none' to skip)")
    ap.add_argument("--read-calibration", action="store_true",
                    help="also run a plain 1 GiB device read (sum), the read-only reference of the byte counters")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain 1 GiB device copies (reference for the HBM byte counters)")
    ap.add_argument("--serve-rho", default="0.5,0.8,0.95", help="comma-separated loads rho of the serving runs")
    ap.add_argument("--only", choices=["gcrodr", "complex", "batch", "ceiling"],
                    help="run one arm by itself and print its JSON (for profiling it)")
    ap.add_argument("--c2-no-pool", action="store_true",
                    help="generate the batch workload's systems in this process (no worker processes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X: a job of this workload fits one GPU and the library does not "
              "shard; --gpus above 1 is not supported (DESIGN.md describes how the path would shard).",
              file=sys.stderr)
        sys.exit(2)

    import tempfile
    tune_file = os.environ.get("PMOR_TUNE_CACHE")
    if tune_file is None:  # record what the library's tuner chooses in this run
        tune_file = os.path.join(tempfile.mkdtemp(prefix="pmor_tune_"), "tune.json")
        os.environ["PMOR_TUNE_CACHE"] = tune_file

    import torch
    from synth import config0, config1
    from paper_1809_06574_amd import Context, Problem, lib as L

    job = config1() if args.workload == "config1" else config0()
    ctx = Context(0)
    dev = ctx.device
    terms = {r: (torch.as_tensor(T.rowptr, device=dev), torch.as_tensor(T.col, device=dev),
                 torch.as_tensor(T.val, device=dev)) for r, T in job.terms.items()}
    B = torch.as_tensor(job.B, device=dev)
    Xbuf = torch.empty((len(job.p_list),) + tuple(B.shape), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def factory():
        return Problem(ctx, terms)

    if args.only:
        if args.only == "gcrodr":
            res = gcrodr_bench(ctx, factory, job, B)
        elif args.only == "complex":
            res = complex_bench(ctx)
        elif args.only == "ceiling":  # the streaming probe at the job's block size, reads 1..32 with 0..2 writes
            cache = {}
            blk = 8 * job.n * _kp(job.k) * len(job.p_list)
            for w in (0, 1, 2):
                for nr in (1, 2, 3, 4, 8, 12, 16, 24, 32):
                    mix_ceiling(ctx, L, blk, nr, w, cache)
            res = {"block_MB": blk / 1e6, "GBps": {f"read{k[1]}_write{k[2]}": v for k, v in cache.items()}}
        else:
            res = c2_bench(ctx, args.c2_systems, pool=not args.c2_no_pool)
        print(json.dumps({"only": args.only, args.only: res}), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.read_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        for _ in range(3):
            float(src.sum())
        del src

    # warmup (also builds every lazily created buffer)
    _note("warmup")
    for _ in range(max(args.warmup, 0)):
        run_job(factory, job, B, "update", Xbuf=Xbuf)

    # the dominant kernel: one untimed job per kernel class, the one with the most device time
    kinds = dict(L.PROF_KERNELS)
    per_kernel = {}
    if args.roofline_kernel == "auto":
        for name, kid in kinds.items():
            L.check(L.pmor_prof_set(ctx.handle, kid), "prof_set")
            run_job(factory, job, B, "update", Xbuf=Xbuf)
            n_, ms_, by_ = _prof_read(L, ctx)
            per_kernel[name] = {"launches": n_, "total_ms": ms_, "avg_us": 1e3 * ms_ / max(n_, 1),
                                "GBps": by_ / max(ms_ * 1e-3, 1e-12) / 1e9}
        dom = max(per_kernel, key=lambda k: per_kernel[k]["total_ms"])
    else:
        dom = args.roofline_kernel

    # timed region: update policy, dominant kernel timed live
    _note(f"timed jobs (dominant kernel {dom})")
    L.check(L.pmor_prof_set(ctx.handle, kinds[dom]), "prof_set")
    lat_upd = []
    t_upd, n_upd = timed(lambda: run_job(factory, job, B, "update", lat=lat_upd, Xbuf=Xbuf), args.steps)
    nl, ms, by = _prof_read(L, ctx)
    L.check(L.pmor_prof_set(ctx.handle, 0), "prof_set")
    achieved = by / (ms * 1e-3) / 1e9
    value = n_upd / t_upd

    out = {"metric": "parametric solves/s at 1e-8 residual (SPAI-update vs rebuild); p50/p99 latency",
           "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t_upd / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{job.name}: 3-D 7-point grid {'x'.join(map(str, job.meta['dims']))}, "
                                  f"n={job.n}, nnz(A)={_nnz(factory)}, k={job.k}, "
                                  f"{len(job.p_list)} points p in [{job.p_list[0]:.2f},{job.p_list[-1]:.2f}], "
                                  f"s={job.s}, block GMRES(30) tol 1e-8, SPAI on pattern(A), update=U-diag",
                      "policy": "update", "execution": "points of a job solved together (pmor_sequence_solve)",
                      "solves_per_step": n_upd // args.steps},
           "latency_ms": {"p50": 1e3 * _pct(lat_upd, 50), "p99": 1e3 * _pct(lat_upd, 99)},
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic(dom), "launches": nl,
                        "avg_launch_us": 1e3 * ms / max(nl, 1),
                        "bytes_per_launch": by / max(nl, 1)},
           }
    ceil = stream_ceiling(ctx, L, dom, 8 * job.n * _kp(job.k) * len(job.p_list), by / max(nl, 1))
    if ceil is not None:
        out["roofline"]["stream_ceiling"] = ceil
        out["roofline"]["frac_of_stream_ceiling"] = achieved / ceil["at_kernel_mix"]
    if per_kernel:
        out["kernels"] = per_kernel

    if not args.no_arms:
        _note("arms")
        arms = {"update_batched": (value, lat_upd)}
        for name, policy, mode, steps in (("rebuild_batched", "rebuild", "batched", args.steps),
                                          ("update_pointwise", "update", "pointwise", 1),
                                          ("rebuild_pointwise", "rebuild", "pointwise", 1),
                                          ("plain_nonblock_rebuild", "rebuild", "plain", 1)):
            run_job(factory, job, B, policy, mode=mode, Xbuf=Xbuf)  # untimed: tunes this path's kernels
            lat = []
            t_a, n_a = timed(lambda: run_job(factory, job, B, policy, mode=mode, lat=lat, Xbuf=Xbuf), steps)
            arms[name] = (n_a / t_a, lat)
        # the second approach of Table 1 (anchor A(l-1)) as an ablation, and the
        # block steps per point of both approaches
        st_first, st_second = [], []
        pb = factory()
        _, sq = pb.sequence_solve(B, [job.s] * len(job.p_list), job.p_list, policy="update", X=Xbuf)
        a1 = float(torch.linalg.norm(pb.assemble(job.s, job.p_list[0])))
        pb.close()
        misfit = [st["fro_resid"] / a1 for st in sq[1:]]  # ||A(1) - A(l) diag(q)||_F / ||A(1)||_F
        run_job(factory, job, B, "update", Xbuf=Xbuf, steps=st_first)
        run_job(factory, job, B, "update", Xbuf=Xbuf, approach="second", steps=st_second)
        lat = []
        t_a, n_a = timed(lambda: run_job(factory, job, B, "update", lat=lat, Xbuf=Xbuf, approach="second"),
                         args.steps)
        arms["update_second_approach_batched"] = (n_a / t_a, lat)
        # the adaptive Q pattern at the paper's MSPAI tolerance (1e-4) and at 0.02
        st_adapt = {}
        for tag, ep in (("1e-4", 1e-4), ("0.02", 0.02)):
            st_adapt[tag] = []
            run_job(factory, job, B, "update", Xbuf=Xbuf, update="adaptive", adapt_ep=ep, steps=st_adapt[tag])
            lat = []
            t_a, n_a = timed(lambda: run_job(factory, job, B, "update", lat=lat, Xbuf=Xbuf, update="adaptive",
                                             adapt_ep=ep), args.steps)
            arms[f"update_adaptive_ep{tag}_batched"] = (n_a / t_a, lat)
        out["arms"] = {k: {"solves_per_s": v, "p50_ms": 1e3 * _pct(l, 50), "p99_ms": 1e3 * _pct(l, 99)}
                       for k, (v, l) in arms.items()}
        out["update_approaches"] = {"steps_per_point_first": st_first, "steps_per_point_second": st_second,
                                    "steps_per_point_adaptive_ep1e-4": st_adapt["1e-4"],
                                    "steps_per_point_adaptive_ep0.02": st_adapt["0.02"],
                                    "first_update_misfit_max": max(misfit) if misfit else 0.0,
                                    "first_update_misfit_last": misfit[-1] if misfit else 0.0}
        _note("block GCRO-DR")
        out["gcrodr_pointwise"] = gcrodr_bench(ctx, factory, job, B)
        out["update_vs_rebuild"] = value / arms["rebuild_batched"][0]
        out["update_vs_plain"] = value / arms["plain_nonblock_rebuild"][0]
        out["batched_vs_pointwise_update"] = value / arms["update_pointwise"][0]

    if not args.no_arms:
        _note("complex points")
        out["complex_points"] = complex_bench(ctx)

    kept = {}
    if not args.no_precisions:
        _note("least-squares precisions")
        npts = len(job.p_list)
        out["precisions"] = c3_bench(factory, job, B, keep_points=(0, npts // 2, npts - 1), kept=kept)

    if args.c2_systems > 0:
        out["batch_systems"] = c2_bench(ctx, args.c2_systems, pool=not args.c2_no_pool)

    if args.serve_jobs > 0:
        _note("serving")
        rhos = [float(x) for x in args.serve_rho.split(",")]
        out["serving"] = serve_bench(ctx, rhos, args.serve_jobs)

    if not args.no_rooflines:
        _note("spai and spmm rooflines")
        out["spai_rooflines"] = spai_rooflines(ctx, L, factory, job)
        if args.spmm_sizes != "none":
            sizes = [tuple(int(v) for v in t.split("x")) for t in args.spmm_sizes.split(",")]
            out["spmm_rooflines"] = spmm_rooflines(ctx, L, sizes)

    if not args.no_cpu_baseline:
        _note("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(job, kept)
        for prec, errs in out["cpu_baseline"].pop("precision_rel_err_vs_oracle_f64").items():
            out["precisions"][prec]["rel_err_vs_oracle_f64"] = errs
    try:
        with open(tune_file) as f:
            out["tuning"] = json.load(f)
    except (OSError, ValueError):
        out["tuning"] = None
    print(json.dumps(out), flush=True)


def serve_bench(ctx, rhos, n_jobs, n_cal=12, alone=5, engine_rows=40_000_000, seed_base=0):
    """Sequence jobs of the serving workload (n uniform over 32x32x16, 64x32x32, 64^3,
    128x128x64; 20 points p0 + 0.02 j; k = 4) arriving as a Poisson process at
    rate rho * mu_hat, served by one pmor_server (continuous batching).  mu_hat =
    jobs/s of the server when n_cal jobs of the same mix arrive together.
    Returns the report dict."""
    import torch
    from synth import config4_job
    from paper_1809_06574_amd import Problem, Server

    import multiprocessing as mp

    dev = ctx.device
    cal = list(range(10_000, 10_000 + n_cal))
    all_ids = cal + list(range(n_jobs))
    # inputs generated and made resident before any timed run
    pool = mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1))
    try:
        jobs = pool.map(config4_job, all_ids)
    finally:
        pool.close()  # let the workers exit on their own (no terminate signal)
        pool.join()
    cache = {}
    for jid, job in zip(all_ids, jobs):
        terms = {r: (torch.as_tensor(T.rowptr, device=dev), torch.as_tensor(T.col, device=dev),
                     torch.as_tensor(T.val, device=dev)) for r, T in job.terms.items()}
        cache[jid] = (job, terms, torch.as_tensor(job.B, device=dev))
    torch.cuda.synchronize()

    def job_dev(jid):
        return cache[jid]

    def run(jids, arrivals, keep=()):
        sv = Server(ctx, k=4, engine_rows=engine_rows, max_systems=128)
        t0 = time.perf_counter()
        nxt, sub, fin, kept, meta = 0, {}, {}, {}, {}
        solve_lat = []
        while len(fin) < len(jids):
            now = time.perf_counter() - t0
            while nxt < len(jids) and arrivals[nxt] <= now:
                job, terms, B = job_dev(jids[nxt])
                t_arr = t0 + arrivals[nxt]
                pb = Problem(ctx, terms)
                jid = sv.submit(pb, B, [job.s] * len(job.p_list), job.p_list)
                sub[jid] = (nxt, t_arr, time.perf_counter(), job.n)
                nxt += 1
            inf = sv.info()
            if inf["queued"] + inf["admitted"] + inf["running"] == 0:
                if nxt < len(jids):
                    time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
                continue
            for jid, status, X, stats in sv.step():
                q, t_arr, t_sub, n = sub[jid]
                fin[q] = (time.perf_counter() - t_arr, status, n)
                solve_lat += [(t_sub - t_arr) + st["t_solve_ms"] * 1e-3 for st in stats]
                if q in keep:
                    kept[q] = X.clone()
        makespan = time.perf_counter() - t0
        sv.close()
        return makespan, fin, solve_lat, kept

    rng = np.random.default_rng(1004 + seed_base)
    mk, _, _, _ = run(cal, [0.0] * n_cal)
    mu_hat = n_cal / mk
    rep = {"mu_hat_jobs_per_s": mu_hat, "calibration": f"{n_cal} jobs of the mix submitted at once: {mk:.2f} s",
           "jobs_per_run": n_jobs, "points_per_job": 20, "k": 4, "rho": {}}
    for rho in rhos:
        lam = rho * mu_hat
        arr = np.cumsum(rng.exponential(1.0 / lam, size=n_jobs))
        arr -= arr[0]
        jids = list(range(n_jobs))
        keep = tuple(range(0, n_jobs, max(1, n_jobs // alone)))[:alone]
        mk, fin, slat, kept = run(jids, list(arr), keep)
        jl = [v[0] for v in fin.values()]
        ok = all(v[1] == 0 for v in fin.values())
        rep["rho"][str(rho)] = {
            "arrival_rate_jobs_per_s": lam, "makespan_s": mk, "all_converged": ok,
            "solves_per_s": 20 * n_jobs / mk, "jobs_per_s": n_jobs / mk,
            "job_latency_ms": {"p50": 1e3 * _pct(jl, 50), "p99": 1e3 * _pct(jl, 99)},
            "solve_latency_ms": {"p50": 1e3 * _pct(slat, 50), "p99": 1e3 * _pct(slat, 99)}}
        if kept:
            same = []
            for q, Xm in kept.items():
                _, _, _, ka = run([jids[q]], [0.0], keep=(0,))
                same.append(bool(torch.equal(ka[0], Xm)))
            rep["rho"][str(rho)]["alone_vs_mix_bitwise"] = {"jobs": len(same), "equal": all(same)}
    cache.clear()
    return rep


def gcrodr_bench(ctx, factory, job, B, configs=((30, 0, "spai"), (30, 8, "spai"), (10, 0, "spai"), (10, 8, "spai"),
                                                 (10, 0, "none"), (10, 8, "none")), none_points=5):
    """The sequence solved point by point with block GCRO-DR (SPAI at the first
    point and the U-diag update, or no preconditioner on the first
    ``none_points`` points), the recycled basis carried from point to point, for
    restart lengths m and recycled dimensions kr (kr = 0: no recycling).  The
    Gram and product kernels are timed live in the (m = 30, kr = 8) run."""
    import torch
    from paper_1809_06574_amd import Recycler, lib as L

    def one(m, kr, prec, prof=0):
        pb = factory()
        rec = Recycler(ctx, job.n, kr)
        X = torch.empty_like(B)
        steps, cyc, rcs = [], [], []
        pts = job.p_list if prec == "spai" else job.p_list[:none_points]
        if prof:
            L.check(L.pmor_prof_set(ctx.handle, prof), "prof_set")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = pb.spai_build(job.s, pts[0]) if prec == "spai" else None
        for l, p in enumerate(pts):
            if l and h is not None:
                h.update(job.s, p)
            _, st, rc = pb.block_solve_gcrodr(h, job.s, p, B, rec, m=m, tol=1e-8, max_cycles=64, X=X,
                                              raise_on_error=False)
            steps.append(st["steps"])
            cyc.append(st["cycles"])
            rcs.append(rc)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        prof_out = None
        if prof:
            prof_out = _prof_read(L, ctx)
            L.check(L.pmor_prof_set(ctx.handle, 0), "prof_set")
        rec.close()
        if h is not None:
            h.close()
        pb.close()
        return t, steps, cyc, rcs, len(pts), prof_out

    one(*configs[0])  # untimed: first-call allocations and kernel loads
    out = {}
    for m, kr, prec in configs:
        t, steps, cyc, rcs, npts, _ = one(m, kr, prec)
        out[f"m{m}_kr{kr}_{prec}"] = {"solves_per_s": npts / t, "points": npts, "steps_per_point": steps,
                                      "cycles_per_point": cyc, "total_steps": sum(steps),
                                      "all_converged": all(r == 0 for r in rcs)}
    kern = {}
    for name, kid in L.PROF_GCRO.items():
        _, _, _, _, _, (nl, ms, by) = one(30, 8, "spai", prof=kid)
        gbs = by / max(ms * 1e-3, 1e-12) / 1e9
        kern[name] = {"launches": nl, "avg_us": 1e3 * ms / max(nl, 1), "GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
                      "bytes_per_launch": by / max(nl, 1)}
    out["kernels_m30_kr8"] = kern
    return out


# (f^2, theta, d) of the complex points on the 64^3 grid: the small job's
# frequencies divided by 100, which keeps them below the lowest resonance of
# the grid's K, M pair (min eig M^-1 K falls with the mesh width squared)
COMPLEX_POINTS_64 = ((2.25e-4, 0.5, 1.0), (2.25e-4, 0.5, 2.0), (2.0e-4, 0.3, 2.0), (1.5e-4, 0.3, 1.5))


def complex_bench(ctx, dims=(64, 64, 64), k=4, steps=3, points=COMPLEX_POINTS_64):
    """The gyroscope-shaped job at four complex points s = 2 pi f sqrt(-1) on a
    dims grid, solved through the equivalent real form (order 2n): the sequence
    with the complex U-diag update, all points together, right-hand sides
    [R(B), R(iB)] (complex block GMRES on k complex columns)."""
    import torch
    from synth import gyro_complex_job
    from paper_1809_06574_amd import Problem
    job = gyro_complex_job(dims=dims, k=k, points=points)
    dev = ctx.device
    terms = [tuple(torch.as_tensor(x, device=dev) for x in (T.rowptr, T.col, T.val)) for T in job.aterms]
    Bc = job.B
    Bh = torch.as_tensor(np.hstack([np.stack([Bc.real, Bc.imag], 1).reshape(2 * job.n, k),
                                    np.stack([-Bc.imag, Bc.real], 1).reshape(2 * job.n, k)]), device=dev)
    pts = [list(c) for c in job.coefs]
    X = torch.empty((len(pts), 2 * job.n, 2 * k), dtype=torch.float64, device=dev)
    pb = Problem(ctx, terms, kinds=job.kinds)
    _, st = pb.sequence_solve(Bh, coefs=pts, X=X)  # untimed: buffers and tuning
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = pb.sequence_solve(Bh, coefs=pts, X=X)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"n_complex": job.n, "n_real_form": pb.n, "nnz_real_form": pb.nnz, "k_complex": k, "points": len(pts),
           "solves_per_s": steps * len(pts) / t, "steps_per_point": [s_["steps"] for s_ in st],
           "relres_max": max(max(s_["relres"]) for s_ in st)}
    # the same points one by one with block GCRO-DR (SPAI at the first point,
    # the complex U-diag update), without and with a recycled subspace
    from paper_1809_06574_amd import Recycler
    for kr in (0, 16):
        rec = Recycler(ctx, pb.n, kr)
        Xp = torch.empty_like(Bh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = pb.spai_build(pts[0], None)
        stp = []
        for l, c in enumerate(pts):
            if l:
                h.update(c)
            _, sg, _ = pb.block_solve_gcrodr(h, c, None, Bh, rec, m=30, tol=1e-8, max_cycles=64, X=Xp)
            stp.append(sg["steps"])
        torch.cuda.synchronize()
        out[f"gcrodr_m30_kr{kr}"] = {"solves_per_s": len(pts) / (time.perf_counter() - t0), "steps_per_point": stp}
        h.close()
        rec.close()
    pb.close()
    return out


def _c2_system(i):
    from synth.gen import config2_system
    return config2_system(i)


def c3_bench(factory, job, B, keep_points=None, kept=None):
    """The C1 job with the SPAI least squares in FP64, FP32 and FP16s (update
    policy, points solved together): throughput, the P_1 build time and its
    residual ||I - A P_1||_F, block steps per point, and how far each X lies
    from the FP64 run's.  kept[prec] receives X at keep_points (host) for the
    comparison with the oracle's FP64 solution."""
    import torch
    npts = len(job.p_list)
    out, ref = {}, None
    for prec in ("f64", "f32", "f16s"):
        def one():
            pb = factory()
            X, st = pb.sequence_solve(B, [job.s] * npts, job.p_list, policy="update", precision=prec)
            pb.close()
            return X, st
        one()  # untimed: this precision's kernels and buffers
        torch.cuda.synchronize()
        t = time.perf_counter()
        X, st = one()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if ref is None:
            ref = X.clone()
        if kept is not None:
            kept[prec] = {l: X[l].cpu().numpy() for l in keep_points}
        dx = max(float(torch.linalg.norm(X[l] - ref[l]) / torch.linalg.norm(ref[l])) for l in range(npts))
        out[prec] = {"solves_per_s": npts / dt, "p1_build_ms": st[0]["t_precond_ms"],
                     "fro_I_minus_AP1": st[0]["fro_resid"],
                     "steps_per_point": sum(sum(s["cycle_steps"]) for s in st) / npts,
                     "max_rel_dX_vs_f64": dx,
                     "max_relres": max(max(s["relres"]) for s in st)}
    return out


def _note(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# blocks each Gram-Schmidt pass writes (kp = 4: pass 2 keeps W' in registers)
SWEEP_WRITES = {"cgs_dot": 0, "cgs_upd_dot": 0, "cgs_upd_gram": 1}
PROBE_READS = (1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 20, 24, 28, 32)


def _kp(k):
    return 1 if k <= 1 else 2 if k <= 2 else 4 if k <= 4 else 8 if k <= 8 else 16


def mix_ceiling(ctx, L, block_bytes, reads, writes, cache):
    """What the chip streams with a kernel's read/write mix (pmor_stream_probe:
    blocks of block_bytes, `writes` of them written): the probe at the two
    allowed read counts around `reads`, interpolated linearly.  Returns
    (GB/s at the mix, {probe key: GB/s})."""
    import ctypes as C
    reads = min(max(reads, PROBE_READS[0]), PROBE_READS[-1])
    lo = max(r for r in PROBE_READS if r <= reads)
    hi = min(r for r in PROBE_READS if r >= reads)
    rates = {}
    for nr in sorted({lo, hi}):
        key = (int(block_bytes), nr, writes)
        if key not in cache:
            us = C.c_double()
            L.check(L.pmor_stream_probe(ctx.handle, nr, writes, int(block_bytes), 10, C.byref(us)),
                    "pmor_stream_probe")
            cache[key] = (nr + writes) * block_bytes / (us.value * 1e-6) / 1e9
        rates[f"read{nr}_write{writes}"] = cache[key]
    a, b = rates[f"read{lo}_write{writes}"], rates[f"read{hi}_write{writes}"]
    at = a if hi == lo else a + (b - a) * (reads - lo) / (hi - lo)
    return at, rates


def stream_ceiling(ctx, L, kernel, block_bytes, bytes_per_launch):
    """The streaming ceiling of a Gram-Schmidt sweep at its own read/write mix
    (None for the other kernels), with the read-only and one-write rates at 8,
    12 and 16 blocks for reference."""
    if kernel not in SWEEP_WRITES:
        return None
    cache = {}
    for nr in (8, 12, 16):
        for w in (0, 1):
            mix_ceiling(ctx, L, block_bytes, nr, w, cache)
    w = SWEEP_WRITES[kernel]
    reads = bytes_per_launch / block_bytes - w
    at, _ = mix_ceiling(ctx, L, block_bytes, reads, w, cache)
    rates = {f"read{k[1]}_write{k[2]}": v for k, v in sorted(cache.items(), key=lambda kv: (kv[0][2], kv[0][1]))}
    return {"unit": "GB/s", "block_MB": block_bytes / 1e6, "rates": rates, "kernel_reads_blocks": reads,
            "kernel_writes_blocks": w, "at_kernel_mix": at}


def c2_bench(ctx, nsys, precision="f32", pool=True):
    """Independent systems of the batch workload (n in [4096, 65536], 2-D/3-D,
    k = 8, power-law SPAI patterns of 5..40 nodes, least squares in FP32): P_1 at
    p, the U-diag update at p + 0.02, then the nsys solves at p + 0.02 together
    (pmor_batch_solve) and one after another (block_solve).  The term matrices,
    patterns and right-hand sides are on the device before any clock starts."""
    import torch
    import multiprocessing as mp
    from paper_1809_06574_amd import Problem, batch_solve

    # the generator runs in fresh interpreters (no fork of a process that holds the GPU)
    _note(f"batch workload: generating {nsys} systems")
    jobs = []
    if pool:
        workers = mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1))
        try:
            for job in workers.imap(_c2_system, range(nsys), chunksize=4):
                jobs.append(job)
                if len(jobs) % 64 == 0:
                    _note(f"batch workload: {len(jobs)}/{nsys} systems generated")
        finally:
            workers.close()
            workers.join()
    else:  # in this process (under a counter-collecting profiler every child process would open the GPU)
        jobs = [_c2_system(i) for i in range(nsys)]
    dev = ctx.device
    dterms, dpats, Bs = [], [], []
    for job in jobs:
        dterms.append({r: tuple(torch.as_tensor(x).to(dev) for x in (T.rowptr, T.col, T.val))
                       for r, T in job.terms.items()})
        dpats.append(tuple(torch.as_tensor(x).to(dev) for x in job.pattern))
        Bs.append(torch.as_tensor(job.B, device=dev))
    from paper_1809_06574_amd import lib as L, spai_build_batch, problem_create_batch, spai_update_batch
    # one system after another: problem, P_1 (spai_build), update
    torch.cuda.synchronize()
    t = time.perf_counter()
    for job, terms, pat in zip(jobs, dterms, dpats):
        pb = Problem(ctx, terms)
        h = pb.spai_build(job.s, job.p_list[0], pattern=pat, precision=precision)
        h.update(job.s, job.p_list[1])
        h.close()
        pb.close()
    torch.cuda.synchronize()
    t_prep_single = time.perf_counter() - t
    # the problems, then every P_1 with the least squares of all systems in
    # shared bucketed launches (spai_build_batch), then the updates
    torch.cuda.synchronize()
    t = time.perf_counter()
    pbs, _, _ = problem_create_batch(ctx, dterms)
    t_problems = time.perf_counter() - t
    bitems = [(pb, job.s, job.p_list[0], pat) for pb, job, pat in zip(pbs, jobs, dpats)]
    hs, _, _ = spai_build_batch(ctx, bitems, precision=precision)
    t_spai = time.perf_counter() - t - t_problems
    spai_update_batch(ctx, [(h, job.s, job.p_list[1]) for job, h in zip(jobs, hs)])
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t
    t_updates = t_prep - t_problems - t_spai
    # the least-squares kernels' own time: the batched P_1 once more under the
    # library's kernel timer
    L.check(L.pmor_prof_set(ctx.handle, L.PROF_KERNELS["spai_ls"]), "prof_set")
    hs2, _, _ = spai_build_batch(ctx, bitems, precision=precision)
    _, ls_ms, _ = _prof_read(L, ctx)
    L.check(L.pmor_prof_set(ctx.handle, 0), "prof_set")
    for h in hs2:
        h.close()
    items = [(pb, h, job.s, job.p_list[1], B) for pb, h, job, B in zip(pbs, hs, jobs, Bs)]
    batch_solve(ctx, items)  # warm the engine buffers
    torch.cuda.synchronize()
    t = time.perf_counter()
    Xs, stats, status, rc = batch_solve(ctx, items)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    t = time.perf_counter()
    for pb, h, job, B in zip(pbs, hs, jobs, Bs):
        pb.block_solve(h, job.s, job.p_list[1], B)
    torch.cuda.synchronize()
    t_point = time.perf_counter() - t
    ns = [job.n for job in jobs]
    # least-squares flops of the P_1 builds, sum over columns of 2 |J|^2 (|I| - |J|/3)
    ls_flops = 0.0
    for h in hs:
        jc, _, ic, _ = h.export_sets()
        nj = torch.diff(jc.to(torch.float64))
        ni = torch.diff(ic.to(torch.float64))
        ls_flops += float(torch.sum(2.0 * nj * nj * (ni - nj / 3.0)))
    out = {"systems": nsys, "n_min": min(ns), "n_max": max(ns), "k": 8, "ls_precision": precision,
           "pattern_sizes": "power law t^-2 on [5, 40]", "all_converged": all(x == 0 for x in status),
           "steps_total": int(sum(st["steps"] for st in stats)),
           "setup_pattern_spai_update_s": t_prep, "setup_problems_s": t_problems,
           "setup_spai_batch_s": t_spai, "setup_updates_s": t_updates,
           "setup_one_system_at_a_time_s": t_prep_single,
           "batched_solves_per_s": nsys / t_batch, "pointwise_solves_per_s": nsys / t_point,
           "batched_solves_per_s_with_setup": nsys / (t_batch + t_prep),
           "setup_ls_gflop": ls_flops / 1e9, "setup_ls_kernel_ms": ls_ms,
           "setup_ls_gflops": ls_flops / max(ls_ms * 1e-3, 1e-12) / 1e9,
           "batched_vs_pointwise": t_point / t_batch}
    for h in hs:
        h.close()
    for pb in pbs:
        pb.close()
    return out


def _traffic(kernel):
    """HBM bytes per launch of the kernel from the committed counter passes
    (profiles/traffic_<kernel>_config1.txt), or None when that file is missing
    or the kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_config1.txt")
    try:
        rec = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
        src = open(os.path.join(ROOT, "paper_1809_06574_amd", "csrc", "krylov.hip"), "rb").read()
        if rec.get("kernel") != kernel or rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _prof_read(L, ctx):
    import ctypes as C
    n, ms, by = C.c_int64(), C.c_double(), C.c_double()
    L.check(L.pmor_prof_read(ctx.handle, C.byref(n), C.byref(ms), C.byref(by)), "prof_read")
    return n.value, ms.value, by.value


def _nnz(factory):
    pb = factory()
    nnz = pb.nnz
    pb.close()
    return nnz


if __name__ == "__main__":
    main()
