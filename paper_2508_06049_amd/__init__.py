"""MI355X-native hierarchical-hybrid-grid full multigrid with the FMG-difference error
estimator (kl-refinement, Mann & Rude).

* ``HHG``        -- one solver context (C-ABI library ``libhhg.so`` built from ``csrc/``)
* ``HHGSolve``   -- torch.autograd.Function whose backward runs the adjoint solve
* ``mesh``       -- host-side coarse-mesh marking and red-green refinement
"""
from ._lib import HHG, HHGError, SolveStats, load, exported_symbols  # noqa: F401
from .autograd import HHGSolve, hhg_solve  # noqa: F401
