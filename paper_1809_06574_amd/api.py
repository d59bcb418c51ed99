"""Thin Python objects over the C ABI, with PyTorch tensors as device memory.

Only argument marshalling happens here: every step of assembly, SPAI,
update and block GMRES runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import types
from typing import Dict, Optional, Sequence

import torch

from . import lib as L


def _dev_i32(x, device):
    return torch.as_tensor(x, dtype=torch.int32).to(device).contiguous()


def _dev_f64(x, device):
    return torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()


def _flat(c, pb):
    """One point's coefficients as the doubles the *_c calls read: a complex
    problem's as (Re, Im) pairs; the count is checked against the problem."""
    if pb.complex:
        vals = [float(v) for x in c for v in (complex(x).real, complex(x).imag)]
    else:
        vals = [float(x) for x in c]
    if len(vals) != pb.ncoef:
        raise ValueError(f"a point of this problem has {pb.ncoef // (2 if pb.complex else 1)} coefficients, "
                         f"got {len(c)}")
    return vals


def _coef(c, pb):
    """A point given as a coefficient vector: a host double array for the *_c calls."""
    vals = _flat(c, pb)
    return (C.c_double * max(len(vals), 1))(*vals)


def _coefs(rows, pb):
    """The points of a sequence, row after row, as one host double array."""
    vals = [v for row in rows for v in _flat(row, pb)]
    return (C.c_double * max(len(vals), 1))(*vals)


def complex_to_real(Bc: torch.Tensor) -> torch.Tensor:
    """An n x k complex block as the 2n x k real block of the equivalent real form
    (row 2i the real parts of row i, row 2i+1 its imaginary parts)."""
    return torch.view_as_real(Bc.to(torch.complex128)).permute(0, 2, 1).reshape(2 * Bc.shape[0], Bc.shape[1])


def real_to_complex(Xr: torch.Tensor) -> torch.Tensor:
    """Inverse of complex_to_real (the last two dimensions; a leading batch dimension is kept)."""
    lead = Xr.shape[:-2]
    n2, k = Xr.shape[-2:]
    v = Xr.reshape(*lead, n2 // 2, 2, k).transpose(-1, -2).contiguous()
    return torch.view_as_complex(v)


def _is_coef(s, p):
    """Points are (s, p), or a coefficient vector passed as s with p None."""
    return p is None


class Context:
    """A device and the HIP stream all calls are ordered on."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        L.check(L.pmor_ctx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)), "pmor_ctx_create")
        self.handle = h

    def close(self):
        if self.handle:
            L.pmor_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _csr_array(terms, affine, dev, keep):
    """The pmor_csr array of a problem's terms (a list, or a dict by role with
    absent roles NULL); the device tensors it points to go into ``keep``."""
    seq = list(terms) if affine else [terms.get(role) for role in L.ROLES]
    csrs = [None] * len(seq)
    for r, T in enumerate(seq):
        if T is None:
            continue
        rp, ci, va = (T.rowptr, T.col, T.val) if hasattr(T, "rowptr") else T
        rp, ci, va = _dev_i32(rp, dev), _dev_i32(ci, dev), _dev_f64(va, dev)
        keep += [rp, ci, va]
        csrs[r] = L.Csr(rp.numel() - 1, ci.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    keep.append(csrs)
    arr = (C.POINTER(L.Csr) * max(len(seq), 1))(*[C.pointer(c) if c is not None else None for c in csrs])
    return seq, arr


class Problem:
    """A parametric system: A(s,p) = s^2 M(p) + s D(p) + K(p) (terms by role, a dict),
    or the affine A(c) = sum_t c_t T_t (terms a list; points are coefficient vectors)."""

    def __init__(self, ctx: Context, terms, kinds=None, _handle=None):
        """``terms[role] = (rowptr, col, val)`` arrays (host or device) or an object with
        ``rowptr``, ``col``, ``val`` attributes; roles M0, M1, D0, D1, K0, K1.  A list
        of such terms makes an affine problem (pmor_problem_create_affine); with
        ``kinds`` (one of "real", "imag", "complex" per term) its coefficients are
        complex and the problem is the equivalent real one of order 2n
        (pmor_problem_create_complex; blocks through complex_to_real)."""
        self.ctx = ctx
        self._keep = []
        self.affine = isinstance(terms, (list, tuple))
        self.complex = kinds is not None
        if self.complex and not self.affine:
            raise ValueError("complex coefficients need a list of terms")
        if _handle is not None:  # made by problem_create_batch
            self.nmaps = self.ncoef = len(terms) if self.affine else len(L.ROLES)
            self._finish(_handle)
            return
        seq, arr = _csr_array(terms, self.affine, ctx.device, self._keep)
        h = C.c_void_p()
        if self.complex:
            kd = {"real": L.PMOR_COEF_REAL, "imag": L.PMOR_COEF_IMAG, "complex": L.PMOR_COEF_COMPLEX}
            if len(kinds) != len(seq):
                raise ValueError("one kind per term")
            ka = (C.c_int32 * len(seq))(*[kd[x] for x in kinds])
            L.check(L.pmor_problem_create_complex(ctx.handle, len(seq), arr, ka, C.byref(h)),
                    "pmor_problem_create_complex")
            self.nmaps = sum(2 if x == "complex" else 1 for x in kinds)
            self.ncoef = 2 * len(seq)
        elif self.affine:
            L.check(L.pmor_problem_create_affine(ctx.handle, len(seq), arr, C.byref(h)), "pmor_problem_create_affine")
            self.nmaps = self.ncoef = len(seq)
        else:
            L.check(L.pmor_problem_create(ctx.handle, arr, C.byref(h)), "pmor_problem_create")
            self.nmaps = self.ncoef = len(seq)
        self._finish(h)

    def _finish(self, h):
        self.handle = h
        self._keep = []  # the library copied the terms
        nn, nz = C.c_int32(), C.c_int32()
        L.check(L.pmor_problem_info(h, C.byref(nn), C.byref(nz)), "pmor_problem_info")
        self.n, self.nnz = nn.value, nz.value

    def close(self):
        if self.handle:
            L.pmor_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- pattern / values -------------------------------------------------
    def pattern(self):
        dev = self.ctx.device
        rp = torch.empty(self.n + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        mp = torch.empty(self.nmaps * max(self.nnz, 1), dtype=torch.int32, device=dev)
        L.check(L.pmor_problem_pattern(self.handle, rp.data_ptr(), ci.data_ptr(), mp.data_ptr()), "pattern")
        return rp, ci[: self.nnz], mp[: self.nmaps * self.nnz].view(self.nmaps, self.nnz)

    def assemble(self, s, p=None) -> torch.Tensor:
        """Values of A at (s, p), or at the coefficient vector s when p is None."""
        out = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=self.ctx.device)
        if _is_coef(s, p):
            L.check(L.pmor_assemble_c(self.handle, _coef(s, self), out.data_ptr()), "pmor_assemble_c")
        else:
            L.check(L.pmor_assemble(self.handle, float(s), float(p), out.data_ptr()), "pmor_assemble")
        return out[: self.nnz]

    def spmm(self, aval: torch.Tensor, X: torch.Tensor, alpha=1.0, beta=0.0, Y=None) -> torch.Tensor:
        k = X.shape[1]
        if Y is None:
            Y = torch.zeros_like(X)
        L.check(L.pmor_spmm(self.handle, aval.data_ptr(), X.data_ptr(), X.stride(0), Y.data_ptr(), Y.stride(0), k,
                            float(alpha), float(beta)), "pmor_spmm")
        return Y

    def table2_norms(self, s1, p1, s2, p2):
        a, b = C.c_double(), C.c_double()
        L.check(L.pmor_table2_norms(self.handle, s1, p1, s2, p2, C.byref(a), C.byref(b)), "pmor_table2_norms")
        return a.value, b.value

    def table2_norms_c(self, coef1, coef2):
        a, b = C.c_double(), C.c_double()
        L.check(L.pmor_table2_norms_c(self.handle, _coef(coef1, self), _coef(coef2, self), C.byref(a), C.byref(b)),
                "pmor_table2_norms_c")
        return a.value, b.value

    def table2_norms_noalloc(self, s1, p1, s2, p2):
        """As table2_norms, through the entry point that allocates no device memory."""
        a, b = C.c_double(), C.c_double()
        L.check(L.pmor_table2_norms_noalloc(self.handle, s1, p1, s2, p2, C.byref(a), C.byref(b)),
                "pmor_table2_norms_noalloc")
        return a.value, b.value

    # --- preconditioner / solve ------------------------------------------
    def spai_build(self, s, p, pattern=None, precision="f64", update="diag", stats=False, approach="first",
                   adapt_ep=0.0):
        """SPAI at (s, p), or at the coefficient vector s when p is None."""
        return Spai(self, s, p, pattern=pattern, precision=precision, update=update, stats=stats,
                    approach=approach, adapt_ep=adapt_ep)

    def spai_import(self, s, p, rowptr, col, val, precision="f64", update="diag", approach="first", adapt_ep=0.0):
        """A preconditioner holding the given P (device CSR), anchored at (s, p) or at the
        coefficient vector s when p is None."""
        return Spai(self, s, p, precision=precision, update=update, approach=approach, adapt_ep=adapt_ep,
                    imported=(rowptr, col, val))

    def block_solve(self, spai, s, p, B: torch.Tensor, m=30, tol=1e-8, max_cycles=20, X=None, raise_on_error=True):
        """Block GMRES at (s, p), or at the coefficient vector s when p is None."""
        n, k = B.shape
        if X is None:
            X = torch.empty((n, k), dtype=torch.float64, device=B.device)
        st = L.Stats()
        o = L.SolveOpts(m, max_cycles, tol)
        sh = spai.handle if spai is not None else None
        if _is_coef(s, p):
            rc = L.block_solve_c(self.handle, sh, _coef(s, self), B.data_ptr(), B.stride(0), k, X.data_ptr(), X.stride(0),
                                 C.byref(o), C.byref(st))
        else:
            rc = L.block_solve(self.handle, sh, float(s), float(p), B.data_ptr(), B.stride(0), k, X.data_ptr(),
                               X.stride(0), C.byref(o), C.byref(st))
        if raise_on_error:
            L.check(rc, "block_solve")
        return X, st.as_dict(), rc

    def block_solve_gcrodr(self, spai, s, p, B: torch.Tensor, recycler: "Recycler", m=30, tol=1e-8, max_cycles=20,
                           X=None, raise_on_error=True):
        """Block GCRO-DR at (s, p) (or the coefficient vector s when p is None), using
        and then updating ``recycler``'s recycled basis."""
        n, k = B.shape
        if X is None:
            X = torch.empty((n, k), dtype=torch.float64, device=B.device)
        st = L.Stats()
        o = L.SolveOpts(m, max_cycles, tol)
        sh = spai.handle if spai is not None else None
        if _is_coef(s, p):
            rc = L.block_solve_gcrodr_c(self.handle, sh, _coef(s, self), B.data_ptr(), B.stride(0), k, X.data_ptr(),
                                        X.stride(0), C.byref(o), recycler.handle, C.byref(st))
        else:
            rc = L.block_solve_gcrodr(self.handle, sh, float(s), float(p), B.data_ptr(), B.stride(0), k,
                                      X.data_ptr(), X.stride(0), C.byref(o), recycler.handle, C.byref(st))
        if raise_on_error:
            L.check(rc, "block_solve_gcrodr")
        return X, st.as_dict(), rc

    def sequence_solve(self, B, s_list: Sequence[float] = None, p_list: Sequence[float] = None, policy="update",
                       pattern=None, precision="f64", update="diag", m=30, tol=1e-8, max_cycles=20, X=None,
                       raise_on_error=True, approach="first", reanchor_tol=0.0, adapt_ep=0.0, coefs=None):
        """The sequence at the points (s_list[l], p_list[l]), or at the rows of ``coefs``."""
        n, k = B.shape
        npts = len(coefs) if coefs is not None else len(p_list)
        if X is None:
            X = torch.empty((npts, n, k), dtype=torch.float64, device=B.device)
        so = _spai_opts(pattern, precision, update, self.ctx.device, self, approach, reanchor_tol, adapt_ep)
        vo = L.SolveOpts(m, max_cycles, tol)
        stats = (L.Stats * npts)()
        pol = L.PMOR_UPDATE if policy == "update" else L.PMOR_REBUILD
        if coefs is not None:
            cf = _coefs(coefs, self)
            rc = L.pmor_sequence_solve_c(self.handle, B.data_ptr(), B.stride(0), k, cf, npts, X.data_ptr(),
                                         X.stride(1), pol, C.byref(so), C.byref(vo), stats)
        else:
            sl = (C.c_double * npts)(*[float(x) for x in s_list])
            pl = (C.c_double * npts)(*[float(x) for x in p_list])
            rc = L.pmor_sequence_solve(self.handle, B.data_ptr(), B.stride(0), k, sl, pl, npts, X.data_ptr(),
                                       X.stride(1), pol, C.byref(so), C.byref(vo), stats)
        if raise_on_error:
            L.check(rc, "pmor_sequence_solve")
            return X, [s.as_dict() for s in stats]
        return X, [s.as_dict() for s in stats], rc


def problem_create_batch(ctx: Context, terms_list, raise_on_error=True):
    """Several real problems at once (pmor_problem_create_batch): each entry of
    ``terms_list`` is what ``Problem`` takes (a dict by role, or a list of affine
    terms).  Returns (list of Problem or None, list of status codes, rc)."""
    n_it = len(terms_list)
    arr = (L.ProblemItem * max(n_it, 1))()
    keep = []
    for i, terms in enumerate(terms_list):
        affine = isinstance(terms, (list, tuple))
        seq, carr = _csr_array(terms, affine, ctx.device, keep)
        keep.append(carr)
        arr[i] = L.ProblemItem(len(seq) if affine else 0, C.cast(carr, C.c_void_p), None, 0)
    rc = L.pmor_problem_create_batch(ctx.handle, arr, n_it)
    out, status = [], []
    for i, terms in enumerate(terms_list):
        status.append(arr[i].status)
        out.append(Problem(ctx, terms, _handle=C.c_void_p(arr[i].pb)) if arr[i].pb else None)
    if raise_on_error:
        L.check(rc, "pmor_problem_create_batch")
    return out, status, rc


def spai_build_batch(ctx: Context, items, precision="f64", update="diag", raise_on_error=True):
    """P_1 of several problems with the least squares of all in shared launches
    (spai_build_batch).  ``items``: ``(problem, s, p)`` or ``(problem, s, p, pattern)``
    with p None meaning s is a coefficient vector.  Returns (list of Spai or None,
    list of status codes, rc)."""
    n_it = len(items)
    arr = (L.SpaiBuildItem * max(n_it, 1))()
    keep = []
    for i, itm in enumerate(items):
        pb, s, p = itm[:3]
        pattern = itm[3] if len(itm) > 3 else None
        holder = types.SimpleNamespace()  # keeps the pattern tensors alive for the call
        o = _spai_opts(pattern, precision, update, ctx.device, holder)
        keep += [o, holder]
        cf = None
        if _is_coef(s, p):
            cf = _coef(s, pb)
            keep.append(cf)
            s, p = 0.0, 0.0
        arr[i] = L.SpaiBuildItem(pb.handle, float(s), float(p),
                                 C.cast(cf, C.POINTER(C.c_double)) if cf is not None else None,
                                 C.cast(C.pointer(o), C.c_void_p), None, 0, -1)
    rc = L.spai_build_batch(ctx.handle, arr, n_it)
    out, status = [], []
    for i, itm in enumerate(items):
        status.append(arr[i].status)
        out.append(Spai(itm[0], None, None, update=update, _handle=C.c_void_p(arr[i].h)) if arr[i].h else None)
    if raise_on_error:
        L.check(rc, "spai_build_batch")
    return out, status, rc


def spai_update_batch(ctx: Context, items, raise_on_error=True):
    """spai_update of several handles, each at its own point (spai_update_batch).
    ``items``: ``(spai, s, p)`` with p None meaning s is a coefficient vector.
    Returns (list of status codes, rc)."""
    n_it = len(items)
    arr = (L.SpaiUpdateItem * max(n_it, 1))()
    keep = []
    for i, (h, s, p) in enumerate(items):
        cf = None
        if _is_coef(s, p):
            cf = _coef(s, h.pb)
            keep.append(cf)
            s, p = 0.0, 0.0
        arr[i] = L.SpaiUpdateItem(h.handle, float(s), float(p),
                                  C.cast(cf, C.POINTER(C.c_double)) if cf is not None else None, 0, -1)
    rc = L.spai_update_batch(ctx.handle, arr, n_it)
    status = [arr[i].status for i in range(n_it)]
    if raise_on_error:
        L.check(rc, "spai_update_batch")
    return status, rc


def batch_solve(ctx: Context, items, m=30, tol=1e-8, max_cycles=20, raise_on_error=True):
    """Solve independent systems together (pmor_batch_solve).  ``items``: sequence of
    ``(problem, spai_or_None, s, p, B)`` or ``(problem, spai, s, p, B, X)``; with p None,
    s is the point's coefficient vector.
    Returns (list of X, list of stats dicts, list of status codes, rc)."""
    n_it = len(items)
    arr = (L.BatchItem * max(n_it, 1))()
    Xs = []
    keep = []
    for i, itm in enumerate(items):
        pb, sp, s, p, B = itm[:5]
        X = itm[5] if len(itm) > 5 and itm[5] is not None else torch.empty(B.shape, dtype=torch.float64,
                                                                              device=B.device)
        Xs.append(X)
        cf = None
        if _is_coef(s, p):
            cf = _coef(s, pb)
            keep.append(cf)
            s, p = 0.0, 0.0
        arr[i] = L.BatchItem(pb.handle, sp.handle if sp is not None else None, float(s), float(p), B.data_ptr(),
                             B.stride(0), B.shape[1], X.data_ptr(), X.stride(0),
                             C.cast(cf, C.POINTER(C.c_double)) if cf is not None else None)
    stats = (L.Stats * max(n_it, 1))()
    status = (C.c_int32 * max(n_it, 1))()
    o = L.SolveOpts(m, max_cycles, tol)
    rc = L.pmor_batch_solve(ctx.handle, arr, n_it, C.byref(o), stats, status)
    if raise_on_error:
        L.check(rc, "pmor_batch_solve")
    return Xs, [stats[i].as_dict() for i in range(n_it)], [status[i] for i in range(n_it)], rc


def _spai_opts(pattern, precision, update, device, keeper, approach="first", reanchor_tol=0.0, adapt_ep=0.0):
    o = L.SpaiOpts()
    o.reanchor_tol = float(reanchor_tol)
    o.adapt_ep = float(adapt_ep)
    o.precision = {"f64": L.PMOR_F64, "f32": L.PMOR_F32, "f16s": L.PMOR_F16S}[precision]
    o.update = {"diag": L.PMOR_UPD_DIAG, "pattern": L.PMOR_UPD_PATTERN, "adaptive": L.PMOR_UPD_ADAPTIVE}[update]
    o.approach = {"first": L.PMOR_APPROACH_FIRST, "second": L.PMOR_APPROACH_SECOND}[approach]
    if pattern is None:
        o.pattern = L.PMOR_PAT_A
    else:
        cp, rw = _dev_i32(pattern[0], device), _dev_i32(pattern[1], device)
        keeper._pat = (cp, rw)
        o.pattern = L.PMOR_PAT_EXPLICIT
        o.nnz_explicit = rw.numel()
        o.pat_colptr = cp.data_ptr()
        o.pat_row = rw.data_ptr()
    return o


class Spai:
    """SPAI of A(s,p) on a pattern, with the update of Table 1 (first approach by
    default; approach="second" anchors each update at the previous point)."""

    def __init__(self, pb: Problem, s, p, pattern=None, precision="f64", update="diag", stats=False,
                 approach="first", adapt_ep=0.0, imported=None, _handle=None):
        self.pb = pb
        self.update_kind = update
        self.approach = approach
        if _handle is not None:  # a handle the library built already (spai_build_batch)
            self.handle = _handle
            self.last_stats = None
            nz, mj, mi = C.c_int32(), C.c_int32(), C.c_int32()
            L.check(L.spai_info(self.handle, C.byref(nz), C.byref(mj), C.byref(mi)), "spai_info")
            self.nnzP, self.maxJ, self.maxI = nz.value, mj.value, mi.value
            return
        o = _spai_opts(pattern, precision, update, pb.ctx.device, self, approach, adapt_ep=adapt_ep)
        h = C.c_void_p()
        st = L.Stats()
        sb = C.byref(st) if stats else None
        if imported is not None:
            rp, ci, va = (t.contiguous() for t in imported)
            args = (ci.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr(), C.byref(o), C.byref(h))
            rc = (L.spai_import_c(pb.handle, _coef(s, pb), *args) if _is_coef(s, p)
                  else L.spai_import(pb.handle, float(s), float(p), *args))
            where = "spai_import"
        elif _is_coef(s, p):
            rc = L.spai_build_c(pb.handle, _coef(s, pb), C.byref(o), C.byref(h), sb)
            where = "spai_build_c"
        else:
            rc = L.spai_build(pb.handle, float(s), float(p), C.byref(o), C.byref(h), sb)
            where = "spai_build"
        self.handle = h if h.value else None
        self.last_stats = st.as_dict() if stats else None
        L.check(rc, where)
        nz, mj, mi = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.spai_info(self.handle, C.byref(nz), C.byref(mj), C.byref(mi)), "spai_info")
        self.nnzP, self.maxJ, self.maxI = nz.value, mj.value, mi.value

    def update(self, s, p=None, stats=False):
        """Update to (s, p), or to the coefficient vector s when p is None."""
        st = L.Stats()
        sb = C.byref(st) if stats else None
        if _is_coef(s, p):
            L.check(L.spai_update_c(self.handle, _coef(s, self.pb), sb), "spai_update_c")
        else:
            L.check(L.spai_update(self.handle, float(s), float(p), sb), "spai_update")
        self.last_stats = st.as_dict() if stats else None
        return self.last_stats

    def rebuild(self, s, p=None, stats=False):
        st = L.Stats()
        sb = C.byref(st) if stats else None
        if _is_coef(s, p):
            L.check(L.spai_rebuild_c(self.handle, _coef(s, self.pb), sb), "spai_rebuild_c")
        else:
            L.check(L.spai_rebuild(self.handle, float(s), float(p), sb), "spai_rebuild")
        self.last_stats = st.as_dict() if stats else None
        return self.last_stats

    def export(self):
        dev = self.pb.ctx.device
        n = self.pb.n
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(self.nnzP, dtype=torch.int32, device=dev)
        va = torch.empty(self.nnzP, dtype=torch.float64, device=dev)
        qlen = n if self.update_kind == "diag" else self.nnzP
        qv = torch.empty(qlen, dtype=torch.float64, device=dev)
        rho = torch.empty(n, dtype=torch.float64, device=dev)
        L.check(L.spai_export(self.handle, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), qv.data_ptr(),
                              rho.data_ptr()), "spai_export")
        return {"rowptr": rp, "col": ci, "val": va, "q": qv, "rho": rho}

    def gather_sums(self):
        """pmor_spai_gather: the sum of every column's gathered block A(I_j, J_j) (anchor values)."""
        out = torch.empty(self.pb.n, dtype=torch.float64, device=self.pb.ctx.device)
        L.check(L.pmor_spai_gather(self.handle, out.data_ptr()), "pmor_spai_gather")
        return out

    def export_sets(self):
        dev = self.pb.ctx.device
        n = self.pb.n
        nI = C.c_int64()
        L.check(L.spai_export_sets(self.handle, None, None, None, None, C.byref(nI)), "spai_export_sets")
        jc = torch.empty(n + 1, dtype=torch.int32, device=dev)
        jr = torch.empty(self.nnzP, dtype=torch.int32, device=dev)
        ic = torch.empty(n + 1, dtype=torch.int64, device=dev)
        ir = torch.empty(max(nI.value, 1), dtype=torch.int32, device=dev)
        L.check(L.spai_export_sets(self.handle, jc.data_ptr(), jr.data_ptr(), ic.data_ptr(), ir.data_ptr(),
                                   C.byref(nI)), "spai_export_sets")
        return jc, jr, ic, ir[: nI.value]

    def close(self):
        if self.handle:
            L.spai_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Recycler:
    """The recycled subspace of block GCRO-DR, carried across solves (pmor_recycle_*)."""

    def __init__(self, ctx: Context, n: int, kr: int):
        self.ctx = ctx
        self.n, self.kr = n, kr
        h = C.c_void_p()
        L.check(L.pmor_recycle_create(ctx.handle, n, kr, C.byref(h)), "pmor_recycle_create")
        self.handle = h

    @property
    def dim(self) -> int:
        kc = C.c_int32()
        L.check(L.pmor_recycle_info(self.handle, C.byref(kc)), "pmor_recycle_info")
        return kc.value

    def reset(self):
        L.check(L.pmor_recycle_reset(self.handle), "pmor_recycle_reset")

    def export(self) -> torch.Tensor:
        kc = self.dim
        U = torch.empty((self.n, max(kc, 1)), dtype=torch.float64, device=self.ctx.device)
        L.check(L.pmor_recycle_export(self.handle, U.data_ptr(), U.stride(0)), "pmor_recycle_export")
        return U[:, :kc]

    def close(self):
        if self.handle:
            L.pmor_recycle_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching of sequence jobs over one persistent engine (pmor_server_*)."""

    def __init__(self, ctx: Context, k: int, hbm_budget: int = 0, engine_rows: int = 0, max_systems: int = 0,
                 update="diag", precision="f64", m=30, tol=1e-8, max_cycles=20, approach="first", adapt_ep=0.0):
        self.ctx = ctx
        so = _spai_opts(None, precision, update, ctx.device, self, approach, adapt_ep=adapt_ep)
        vo = L.SolveOpts(m, max_cycles, tol)
        opts = L.ServerOpts(int(hbm_budget), int(engine_rows), int(k), int(max_systems))
        h = C.c_void_p()
        L.check(L.pmor_server_create(ctx.handle, C.byref(opts), C.byref(so), C.byref(vo), C.byref(h)),
                "pmor_server_create")
        self.handle = h
        self.jobs = {}

    def submit(self, pb: Problem, B: torch.Tensor, s_list=None, p_list=None, policy="update", X=None, coefs=None):
        """Queue a job at the points (s_list, p_list) or the rows of ``coefs``; returns its id.
        X (npts, n, k) is written when the job is reported done."""
        n, k = B.shape
        npts = len(coefs) if coefs is not None else len(p_list)
        if X is None:
            X = torch.empty((npts, n, k), dtype=torch.float64, device=B.device)
        if coefs is not None:
            cf = _coefs(coefs, pb)
            sl = pl = None
        else:
            cf = None
            sl = (C.c_double * npts)(*[float(x) for x in s_list])
            pl = (C.c_double * npts)(*[float(x) for x in p_list])
        stats = (L.Stats * npts)()
        pol = L.PMOR_UPDATE if policy == "update" else L.PMOR_REBUILD
        job = L.Job(pb.handle, B.data_ptr(), B.stride(0), k, sl, pl, npts, X.data_ptr(), X.stride(1), pol, stats,
                    C.cast(cf, C.POINTER(C.c_double)) if cf is not None else None)
        jid = C.c_int64()
        L.check(L.pmor_server_submit(self.handle, C.byref(job), C.byref(jid)), "pmor_server_submit")
        self.jobs[jid.value] = {"pb": pb, "B": B, "X": X, "stats": stats, "s": sl, "p": pl}
        return jid.value

    def step(self, max_done: int = 256):
        """One scheduling round; returns [(job_id, status, X, stats dicts)] of finished jobs."""
        ids = (C.c_int64 * max_done)()
        sts = (C.c_int32 * max_done)()
        nd = C.c_int32()
        L.check(L.pmor_server_step(self.handle, ids, sts, max_done, C.byref(nd)), "pmor_server_step")
        out = []
        for i in range(nd.value):
            rec = self.jobs.pop(ids[i])
            out.append((ids[i], sts[i], rec["X"], [s.as_dict() for s in rec["stats"]]))
        return out

    def info(self):
        q, a, r, b = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        L.check(L.pmor_server_info(self.handle, C.byref(q), C.byref(a), C.byref(r), C.byref(b)), "pmor_server_info")
        return {"queued": q.value, "admitted": a.value, "running": r.value, "bytes": b.value}

    def close(self):
        if self.handle:
            L.pmor_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
