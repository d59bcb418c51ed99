"""CPU oracle for preconditioned parametric linear solves — TEST INFRASTRUCTURE.

A plain, slow, FP64 NumPy implementation of what the GPU library computes,
written from the paper (Singh & Ahuja, "Preconditioned Linear Solves for
Parametric Model Order Reduction"):

* ``assemble``  A(s,p) = s^2 M(p) + s D(p) + K(p) on the union pattern
                (Section 1.1, frequency-domain form; Section 1.2, eq. loewner_eq2).
* ``spai``      SPAI: min ||I - A P||_F split into one least-squares problem per
                column (Section 2.2), solved by Householder QR.
* ``update``    the cheap SPAI update, first approach: min ||A(1) - A(l) Q||_F,
                P_l = Q P_1 (Section 2.3, Table 1; Section 2.4); second approach
                as an ablation (Table 1, right column); the adaptive Q pattern
                and the re-anchoring plan (readings where the paper is silent).
* ``gmres``     block GMRES(m) with right preconditioning (Section 2.1 and its
                footnote on right preconditioning).
* ``diagnostics`` the norms of Table 2 and ||I - A P||_F.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path;
both consume the seeded inputs of the ``synth`` package.  Each function is
pinned by a CPU test against something other than itself (closed forms,
brute force, textbook library routines); see ``tests/test_oracle_*.py``.
"""
from . import sparse, assemble, spai, update, gmres, diagnostics  # noqa: F401
