"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package builds matrices and intervals only; it holds none of the FEAST
arithmetic (no contour, no solve, no Rayleigh-Ritz), so both the HIP path and
the oracle can be fed from it without sharing any of the method's code.
"""

from .generators import (
    helloworld,
    laplacian_1d_dense,
    laplacian_1d_eigs,
    prescribed_complex_pencil,
    prescribed_real_problem,
    batched_real_problems,
    column_major,
    laplacian_3d_csr,
    laplacian_3d_eigs,
    differentiation_problem,
)

__all__ = [
    "helloworld",
    "laplacian_1d_dense",
    "laplacian_1d_eigs",
    "prescribed_complex_pencil",
    "prescribed_real_problem",
    "batched_real_problems",
    "column_major",
    "laplacian_3d_csr",
    "laplacian_3d_eigs",
    "differentiation_problem",
]
