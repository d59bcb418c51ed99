"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds no arithmetic of the method itself (no assembly of
A(s,p), no preconditioner, no solver): it only draws the sparse terms
M, D, K of a parametric second-order system (paper, Section 1, eq. (1)),
right-hand-side blocks and parameter lists, with fixed seeds.
"""
from .gen import (  # noqa: F401
    CSR,
    Job,
    ROLES,
    grid_laplacian,
    config0,
    config1,
    config2_system,
    config4_job,
    appendix1,
    tiny_random_job,
    gyro_like_job,
    gyro_coefs,
    gyro_complex_job,
)
