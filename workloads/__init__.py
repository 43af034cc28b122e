"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds *inputs only*: finite-difference operators in CSR form and
seeded random vectors.  It contains none of the Krylov method's arithmetic, so
that the CPU oracle and the HIP path can both consume it without sharing any
part of the computation they are compared on.

The paper's own workloads (FEM convection-diffusion and membrane matrices,
graph Laplacians; Section 5) are not available, so these finite-difference
operators stand in for them: same structure (sparse PDE operators, 5- and
7-point stencils, non-symmetric convection), with sizes chosen per workload.
"""
from .operators import (CSR, laplacian_2d, anisotropic_2d, convdiff_3d,
                        shifted_laplacian_3d, ragged_laplacian_sizes, stencil_csr)
from .vectors import gaussian_vector, unit_direction

__all__ = ["CSR", "laplacian_2d", "anisotropic_2d", "convdiff_3d", "shifted_laplacian_3d",
           "ragged_laplacian_sizes", "stencil_csr", "gaussian_vector", "unit_direction"]
