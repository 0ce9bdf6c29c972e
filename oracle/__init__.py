"""CPU oracle for the hierarchical-hybrid-grid full-multigrid solve, its error estimator and
the adjoint gradient.

TEST INFRASTRUCTURE ONLY.  This package is imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py`` -- nothing in the product package imports,
links or executes it.  It shares no code with the HIP library: it builds every fine level by
recursive refinement of each macro element (2D: 4-split at edge midpoints; 3D: Bey's eight
children), assembles global sparse matrices element by element, and runs a textbook FMG on
them in float64.

Parity status per function (what pins it is listed in the tests):
  refine.*      pinned: DoF-count formula, volume sum, lattice equality, congruence classes
  assemble.*    pinned: symmetry, zero row sums, affine kernel, closed-form stencils,
                Galerkin identities, 1^T M 1 = |Omega|
  fmg.*         pinned: direct sparse solve, MMS O(h^2) rates, linearity of MG
  estimate.*    pinned: brute-force quadrature, affine special case, effectivity bounds
                (Theorem on eta_j bounds, closed forms reproduced from Tables 1-2)
  estimate.*    (norm variants) pinned: gradient quadrature of the energy norm, mass-matrix
                row sums, Galerkin orthogonality of the energy estimate
  adjoint.*     pinned: duality J = g^T u = lambda^T b, finite differences
  transfer.*    pinned: affine functions exact, nested transfer equals the prolongation
  fmg.refined_cycle / vcycle_lowp (the float32-refined form: float64 residual, float32
                V-cycle on the correction, float64 update) pinned: equals the float64 cycle
                to round-off when run in float64; its float32 correction is the float64 one
                within float32 rounding; its fixed point is the direct solve; it contracts
                like the float64 cycle
"""
from .refine import Hierarchy, build_hierarchy
from . import assemble, colour, fmg, estimate, adjoint, transfer

__all__ = ["Hierarchy", "build_hierarchy", "assemble", "colour", "fmg", "estimate", "adjoint", "transfer"]
