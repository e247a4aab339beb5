"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only builds test problems: sparse matrices from finite-difference
discretisations, non-overlapping partitions, right-hand sides and seeds.  It
contains none of the preconditioner's arithmetic (no subdomain growth, no
splitting, no eigenproblems, no Krylov method), so that the oracle and the HIP
path can both consume it without sharing any of the method.

Conventions (all grids):
  * unknowns sit at the interior nodes of a uniform grid on the unit square or
    cube, h = 1/(m+1), homogeneous Dirichlet boundary values eliminated;
  * lexicographic numbering with x fastest: idx = i + m*j (+ m*m*k);
  * every row is multiplied by h^2 (relative residuals are unaffected);
  * exact zeros are never stored; column indices are sorted within each row.

The paper's own test matrices (SuiteSparse, FreeFEM SUPG meshes, Section 4)
are not available; the problems below stand in for them with the shapes and
structure of the workloads the method is measured on.
"""
from .problems import (  # noqa: F401
    CSR,
    laplace2d,
    convdiff2d,
    convdiff2d_central,
    convdiff2d_complex,
    magnetic_laplace2d,
    convdiff3d,
    diffusion2d_lognormal,
    lognormal2d_values_torch,
    diffusion3d_blocks,
    gaussian_field_2d,
    strip_partition,
    block_partition_2d,
    block_partition_3d,
    bfs_seeds_3d,
    rhs,
    config,
    CONFIGS,
)
