"""MI355X (gfx950) library for preconditioned parametric linear solves.

SPAI preconditioner, its cheap first-approach update and block GMRES for the
sequences A(s, p_j) X = B of parametric model order reduction (Singh & Ahuja,
"Preconditioned Linear Solves for Parametric Model Order Reduction").

``lib`` is the raw C ABI (include/pmor_spai.h); ``Context``, ``Problem`` and
``Spai`` wrap it with PyTorch tensors as device memory.  Importing this
package fails when libpmorspai.so has not been built.
"""
from . import lib  # noqa: F401  (raises ImportError when the HIP library is missing)
from .api import Context, Problem, Spai  # noqa: F401
