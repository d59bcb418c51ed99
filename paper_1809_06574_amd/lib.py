"""ctypes binding of libpmorspai.so (argument marshalling only).

Every function of include/pmor_spai.h is exposed under its own name with
argtypes set; the shared library must have been built (``build.py``).
Importing this module raises ImportError when it has not.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PMOR_LIB", os.path.join(HERE, "libpmorspai.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_06574_amd.build`")

_lib = C.CDLL(LIB_PATH)

# constants (mirror of the header)
PMOR_OK, PMOR_EINVAL, PMOR_ENOMEM, PMOR_ENOTCONV = 0, -1, -2, -3
PMOR_EBREAKDOWN, PMOR_ESINGULAR, PMOR_ENAN, PMOR_EHIP, PMOR_EADMIT = -4, -5, -6, -7, -8
PMOR_KMAX = 16
PMOR_NROLES = 6
PMOR_TMAX = 16
PMOR_COEF_REAL, PMOR_COEF_IMAG, PMOR_COEF_COMPLEX = 0, 1, 2
PMOR_MAX_CYCLES = 64
ROLES = ("M0", "M1", "D0", "D1", "K0", "K1")
PMOR_PAT_A, PMOR_PAT_EXPLICIT = 0, 1
PMOR_F64, PMOR_F32, PMOR_F16S = 0, 1, 2
PMOR_UPD_DIAG, PMOR_UPD_PATTERN, PMOR_UPD_ADAPTIVE = 0, 1, 2
PMOR_REBUILD, PMOR_UPDATE = 0, 1
PMOR_APPROACH_FIRST, PMOR_APPROACH_SECOND = 0, 1
PROF_KERNELS = {"spmm_a": 1, "cgs_upd_dot": 2, "cgs_dot": 3, "spai_ls": 4, "spmm_p": 5, "cgs_upd_gram": 6}
PROF_SPAI_GATHER = 7
PROF_GCRO = {"gcro_gram": 8, "gcro_gemm": 9}


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class SpaiOpts(C.Structure):
    _fields_ = [("pattern", C.c_int32), ("precision", C.c_int32), ("update", C.c_int32),
                ("nnz_explicit", C.c_int32), ("pat_colptr", C.c_void_p), ("pat_row", C.c_void_p),
                ("approach", C.c_int32), ("reanchor_tol", C.c_double), ("adapt_ep", C.c_double)]


class SpaiBuildItem(C.Structure):
    _fields_ = [("pb", C.c_void_p), ("s", C.c_double), ("p", C.c_double), ("coef", C.POINTER(C.c_double)),
                ("opts", C.c_void_p), ("h", C.c_void_p), ("status", C.c_int32), ("bad_column", C.c_int32)]


class SpaiUpdateItem(C.Structure):
    _fields_ = [("h", C.c_void_p), ("s", C.c_double), ("p", C.c_double), ("coef", C.POINTER(C.c_double)),
                ("status", C.c_int32), ("bad_column", C.c_int32)]


class ProblemItem(C.Structure):
    _fields_ = [("nterms", C.c_int32), ("terms", C.c_void_p), ("pb", C.c_void_p), ("status", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("max_cycles", C.c_int32), ("tol", C.c_double)]


class BatchItem(C.Structure):
    _fields_ = [("pb", C.c_void_p), ("h", C.c_void_p), ("s", C.c_double), ("p", C.c_double),
                ("B", C.c_void_p), ("ldb", C.c_int64), ("k", C.c_int32), ("X", C.c_void_p), ("ldx", C.c_int64),
                ("coef", C.POINTER(C.c_double))]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("engine_rows", C.c_int64), ("k", C.c_int32), ("max_systems", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("k", C.c_int32), ("cycles", C.c_int32), ("steps", C.c_int32), ("bad_column", C.c_int32),
                ("cycle_steps", C.c_int32 * PMOR_MAX_CYCLES), ("relres", C.c_double * PMOR_KMAX),
                ("fro_resid", C.c_double), ("t_assemble_ms", C.c_double), ("t_precond_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("anchor", C.c_int32)]

    def as_dict(self):
        return {"k": self.k, "cycles": self.cycles, "steps": self.steps, "bad_column": self.bad_column,
                "cycle_steps": list(self.cycle_steps[: max(self.cycles, 0)]),
                "relres": list(self.relres[: self.k]), "fro_resid": self.fro_resid,
                "t_assemble_ms": self.t_assemble_ms, "t_precond_ms": self.t_precond_ms,
                "t_solve_ms": self.t_solve_ms, "anchor": self.anchor}


P = C.c_void_p
I32, I64, D = C.c_int32, C.c_int64, C.c_double
PP = C.POINTER(C.c_void_p)


class Job(C.Structure):
    _fields_ = [("pb", C.c_void_p), ("B", C.c_void_p), ("ldb", C.c_int64), ("k", C.c_int32),
                ("s_list", C.POINTER(C.c_double)), ("p_list", C.POINTER(C.c_double)), ("npts", C.c_int32),
                ("X", C.c_void_p), ("ldx", C.c_int64), ("policy", C.c_int32), ("stats", C.POINTER(Stats)),
                ("coefs", C.POINTER(C.c_double))]


_SIGS = {
    "pmor_ctx_create": (C.c_int, [PP, C.c_int, P]),
    "pmor_ctx_destroy": (None, [P]),
    "pmor_ctx_set_stream": (C.c_int, [P, P]),
    "pmor_problem_create": (C.c_int, [P, C.POINTER(C.POINTER(Csr)), PP]),
    "pmor_problem_create_affine": (C.c_int, [P, I32, C.POINTER(C.POINTER(Csr)), PP]),
    "pmor_problem_create_complex": (C.c_int, [P, I32, C.POINTER(C.POINTER(Csr)), C.POINTER(I32), PP]),
    "pmor_problem_destroy": (None, [P]),
    "pmor_problem_info": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32)]),
    "pmor_problem_pattern": (C.c_int, [P, P, P, P]),
    "pmor_assemble": (C.c_int, [P, D, D, P]),
    "pmor_assemble_c": (C.c_int, [P, C.POINTER(D), P]),
    "spai_build": (C.c_int, [P, D, D, C.POINTER(SpaiOpts), PP, C.POINTER(Stats)]),
    "spai_build_c": (C.c_int, [P, C.POINTER(D), C.POINTER(SpaiOpts), PP, C.POINTER(Stats)]),
    "spai_build_batch": (C.c_int, [P, C.POINTER(SpaiBuildItem), I32]),
    "pmor_problem_create_batch": (C.c_int, [P, C.POINTER(ProblemItem), I32]),
    "spai_update_batch": (C.c_int, [P, C.POINTER(SpaiUpdateItem), I32]),
    "spai_update": (C.c_int, [P, D, D, C.POINTER(Stats)]),
    "spai_update_c": (C.c_int, [P, C.POINTER(D), C.POINTER(Stats)]),
    "spai_rebuild": (C.c_int, [P, D, D, C.POINTER(Stats)]),
    "spai_rebuild_c": (C.c_int, [P, C.POINTER(D), C.POINTER(Stats)]),
    "spai_import": (C.c_int, [P, D, D, I32, P, P, P, C.POINTER(SpaiOpts), PP]),
    "spai_import_c": (C.c_int, [P, C.POINTER(D), I32, P, P, P, C.POINTER(SpaiOpts), PP]),
    "spai_info": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]),
    "spai_export": (C.c_int, [P, P, P, P, P, P]),
    "spai_export_sets": (C.c_int, [P, P, P, P, P, C.POINTER(I64)]),
    "spai_free": (None, [P]),
    "block_solve": (C.c_int, [P, P, D, D, P, I64, I32, P, I64, C.POINTER(SolveOpts), C.POINTER(Stats)]),
    "block_solve_c": (C.c_int, [P, P, C.POINTER(D), P, I64, I32, P, I64, C.POINTER(SolveOpts), C.POINTER(Stats)]),
    "pmor_recycle_create": (C.c_int, [P, I32, I32, PP]),
    "pmor_recycle_destroy": (None, [P]),
    "pmor_recycle_info": (C.c_int, [P, C.POINTER(I32)]),
    "pmor_recycle_reset": (C.c_int, [P]),
    "pmor_recycle_export": (C.c_int, [P, P, I64]),
    "block_solve_gcrodr": (C.c_int, [P, P, D, D, P, I64, I32, P, I64, C.POINTER(SolveOpts), P, C.POINTER(Stats)]),
    "block_solve_gcrodr_c": (C.c_int, [P, P, C.POINTER(D), P, I64, I32, P, I64, C.POINTER(SolveOpts), P,
                                       C.POINTER(Stats)]),
    "pmor_harmonic_ritz": (C.c_int, [I32, I32, C.POINTER(D), C.POINTER(D), I32, C.POINTER(D), C.POINTER(D),
                                     C.POINTER(D), C.POINTER(I32)]),
    "pmor_batch_solve": (C.c_int, [P, C.POINTER(BatchItem), I32, C.POINTER(SolveOpts), C.POINTER(Stats),
                                   C.POINTER(I32)]),
    "pmor_sequence_solve": (C.c_int, [P, P, I64, I32, P, P, I32, P, I64, I32, C.POINTER(SpaiOpts),
                                      C.POINTER(SolveOpts), C.POINTER(Stats)]),
    "pmor_sequence_solve_c": (C.c_int, [P, P, I64, I32, C.POINTER(D), I32, P, I64, I32, C.POINTER(SpaiOpts),
                                        C.POINTER(SolveOpts), C.POINTER(Stats)]),
    "pmor_server_create": (C.c_int, [P, C.POINTER(ServerOpts), C.POINTER(SpaiOpts), C.POINTER(SolveOpts), PP]),
    "pmor_server_destroy": (None, [P]),
    "pmor_server_submit": (C.c_int, [P, C.POINTER(Job), C.POINTER(I64)]),
    "pmor_server_step": (C.c_int, [P, C.POINTER(I64), C.POINTER(I32), I32, C.POINTER(I32)]),
    "pmor_server_info": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I64)]),
    "pmor_table2_norms": (C.c_int, [P, D, D, D, D, C.POINTER(D), C.POINTER(D)]),
    "pmor_table2_norms_c": (C.c_int, [P, C.POINTER(D), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    "pmor_table2_norms_noalloc": (C.c_int, [P, D, D, D, D, C.POINTER(D), C.POINTER(D)]),
    "pmor_spmm": (C.c_int, [P, P, P, I64, P, I64, I32, D, D]),
    "pmor_spai_gather": (C.c_int, [P, P]),
    "pmor_prof_set": (C.c_int, [P, C.c_int]),
    "pmor_prof_read": (C.c_int, [P, C.POINTER(I64), C.POINTER(D), C.POINTER(D)]),
    "pmor_stream_probe": (C.c_int, [P, I32, I32, I64, I32, C.POINTER(D)]),
    "pmor_strerror": (C.c_char_p, [C.c_int]),
    "pmor_last_error": (C.c_char_p, []),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class PmorError(RuntimeError):
    def __init__(self, code, where):
        msg = pmor_last_error().decode(errors="replace")
        super().__init__(f"{where}: {pmor_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code, where):
    if code != PMOR_OK:
        raise PmorError(code, where)
    return code


def exported_symbols():
    return sorted(_SIGS)
