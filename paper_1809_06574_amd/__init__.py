"""MI355X (gfx950) library for preconditioned parametric linear solves.

SPAI preconditioner, its cheap update (first approach by default; the second
approach, an adaptive Q pattern and re-anchoring as options) and block GMRES for the
sequences A(s, p_j) X = B of parametric model order reduction (Singh & Ahuja,
"Preconditioned Linear Solves for Parametric Model Order Reduction").

``lib`` is the raw C ABI (include/pmor_spai.h); ``Context``, ``Problem`` and
``Spai`` wrap it with PyTorch tensors as device memory.  They are loaded on
first use, which raises ImportError when libpmorspai.so has not been built
(``python -m paper_1809_06574_amd.build``); there is no fallback path.
"""
import importlib

_LAZY = {"lib": ("lib", None), "Context": ("api", "Context"), "Problem": ("api", "Problem"),
         "Spai": ("api", "Spai"), "batch_solve": ("api", "batch_solve"),
         "Server": ("api", "Server"), "Recycler": ("api", "Recycler"),
         "spai_build_batch": ("api", "spai_build_batch"),
         "problem_create_batch": ("api", "problem_create_batch"),
         "spai_update_batch": ("api", "spai_update_batch"),
         "complex_to_real": ("api", "complex_to_real"), "real_to_complex": ("api", "real_to_complex")}


def __getattr__(name):
    if name not in _LAZY:
        raise AttributeError(name)
    mod, attr = _LAZY[name]
    m = importlib.import_module(f"{__name__}.{mod}")
    return m if attr is None else getattr(m, attr)
