"""Shared helpers of the GPU tests (GPU library vs CPU oracle on the same seeded inputs)."""
import numpy as np

from oracle.sparse import to_scipy


def np_(t):
    return t.detach().cpu().numpy()


def ctx():
    from paper_1809_06574_amd import Context
    return Context(0)


def col_rel_err(n, J_colptr, slot, got, want):
    """max over columns j of ||got_j - want_j|| / ||want_j|| (values in P's CSR order)."""
    worst = 0.0
    for j in range(n):
        s = slot[J_colptr[j]:J_colptr[j + 1]]
        d = np.linalg.norm(got[s] - want[s])
        w = np.linalg.norm(want[s])
        worst = max(worst, d / w if w > 0 else d)
    return worst


def gpu_P_apply(exp, n, update_kind="diag", q_active=False):
    """The preconditioner the GPU applies, as a function X -> P X (from spai_export)."""
    P = to_scipy(n, np_(exp["rowptr"]), np_(exp["col"]), np_(exp["val"]))
    if update_kind == "pattern" and q_active:
        Q = to_scipy(n, np_(exp["rowptr"]), np_(exp["col"]), np_(exp["q"]))
        return lambda X: Q @ (P @ X)
    return lambda X: P @ X
