"""Child process of test_spmm_variants: solves a fixed set of systems (block
widths 1 to 16; preconditioner kinds identity, P_1, diag(q) P_1, Q P_1; a
power-law SPAI pattern) twice, with the engine's sliced-ELL views and with the
CSR arrays, under the SpMM variant that PMOR_SPMM_LPR pins, and saves every X.

usage: python tests/_spmm_worker.py OUT.npz
"""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from synth import config0, tiny_random_job  # noqa: E402
from synth.gen import Job, _nearest_pattern, _power_law_sizes, _weighted_mdk  # noqa: E402


def jobs():
    out = [tiny_random_job(300, 0.02, 11, k=1), tiny_random_job(515, 0.012, 12, k=2), config0(k=3),
           tiny_random_job(333, 0.02, 22, k=8), tiny_random_job(260, 0.03, 23, k=13)]
    rng = np.random.default_rng([2024, 77])
    terms = _weighted_mdk((19, 17, 1), rng, 1e-3)
    K = terms["K0"]
    pat = _nearest_pattern(K, _power_law_sizes(rng, K.n))
    out.append(Job("powerlaw", K.n, terms, 2.0, np.array([0.4, 0.42]), rng.standard_normal((K.n, 8)), pattern=pat))
    return out


def main(path):
    from paper_1809_06574_amd import Context, Problem
    ctx = Context(0)
    res = {}
    for fmt, fill in (("sell", "2"), ("csr", "0")):
        os.environ["PMOR_SELL_MAX_FILL"] = fill
        for i, job in enumerate(jobs()):
            pb = Problem(ctx, job.terms)
            B = torch.as_tensor(job.B, device="cuda")
            s, p0, p1 = job.s, job.p_list[0], job.p_list[1]
            upd = "pattern" if i == 1 else "diag"
            pat = getattr(job, "pattern", None)
            h = pb.spai_build(s, p0, pattern=pat, update=upd)
            X, _, _ = pb.block_solve(h, s, p0, B)  # P_1
            res[f"{fmt}_{i}_p1"] = X.cpu().numpy()
            h.update(s, p1)  # diag(q) P_1, or Q P_1 for the pattern update
            X, _, _ = pb.block_solve(h, s, p1, B)
            res[f"{fmt}_{i}_upd"] = X.cpu().numpy()
            X, _, _ = pb.block_solve(None, s, p1, B)  # no preconditioner
            res[f"{fmt}_{i}_none"] = X.cpu().numpy()
            h.close()
            pb.close()
    np.savez(path, **res)
    print("saved", len(res), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
