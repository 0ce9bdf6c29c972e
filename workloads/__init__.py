"""Seeded, synthetic inputs shared by the oracle tests, the GPU parity tests and the benchmark.

This package holds *inputs only*: coarse macro meshes (vertex coordinates and cell vertex
lists), analytic right-hand sides / boundary data / coefficients, and seeded random
parameters.  It contains none of the multigrid, estimator or adjoint arithmetic, so both the
oracle and the HIP library can consume it without sharing any method code.
"""
from .meshes import (unit_square_2tri, unit_square_grid, lshape_6tri, kuhn_cube,
                     CoarseMesh)
from . import problems

__all__ = ["CoarseMesh", "unit_square_2tri", "unit_square_grid", "lshape_6tri", "kuhn_cube",
           "problems"]
