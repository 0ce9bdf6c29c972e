"""The five workloads the library is measured and checked on, with their synthetic inputs.

All data are analytic or seeded (no dataset exists for this method):
  1  unit square, 2 macro triangles, L=5 (1089 DoFs), u = sin(pi x) sin(pi y), red-black GS,
     FMG with one V(2,2) per level, estimator per macro.
  2  L-shape (-1,1)^2 minus a quadrant, 6 macro triangles k-refined 6 times towards the
     re-entrant corner (144 macros), L=9, u = r^(2/3) sin(2 phi/3) as Dirichlet data, f = 0,
     multicolour GS; float64 and float32-refined; the estimate drives one more k-step.
  3  unit cube, 6 Kuhn tetrahedra, L=7 (129^3 DoFs), kappa = 1 + sin(2 pi x) sin(2 pi y)
     sin(2 pi z)/2 (nodal), Fourier right-hand side (8 modes per axis, N(0,1) amplitudes,
     seed 0), g = 0, red-black GS, float32-refined to a relative residual of 1e-10.
  4  unit cube with the point singularity u = |x|^(1/4) at the corner (0,0,0): the 2^3 Kuhn
     cube (48 tets) k-refined by 3D red-green towards the corner (five steps, each marking the
     12.5 % of macros whose centroids are nearest the corner: 4334 macros), L=5, multicolour.
  5  cube of 4^3 Kuhn cubes (384 tets), L=6 (257^3 DoFs), kappa_e ~ U[0.5, 2] (seed 55),
     Fourier right-hand side (seed 5), goal J(u) = int w u with a Gaussian w (centre
     (1/2,1/2,1/2), sigma 0.1), adjoint gradients.
  6  the mesh and right-hand side of 3 with kappa = 1 per macro, red-black GS: the size scan of
     the smoother bandwidth at L = 8 (257^3) and L = 9 (513^3 DoFs, 135 M).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from workloads import meshes, problems
from workloads.meshes import CoarseMesh

from . import mesh as hostmesh


@dataclass
class Workload:
    name: str
    mesh: CoarseMesh
    L: int
    smoother: str
    f: Callable
    g: Callable
    u_exact: Optional[Callable] = None
    coefficient: str = "macro"
    kappa_cell: Optional[np.ndarray] = None
    kappa_nodal: Optional[Callable] = None
    nu: int = 1
    pre: int = 2
    post: int = 2
    goal_weight: Optional[Callable] = None
    note: str = ""
    extra: dict = field(default_factory=dict)


def _corner_refined_cube(target_steps=(0.125,) * 5) -> CoarseMesh:
    rg = hostmesh.RedGreen3D(meshes.kuhn_cube(2))
    cells, _ = rg.conforming()
    for frac in target_steps:
        X = np.array(rg.X)
        cen = np.array([X[list(c)].mean(0) for c in cells])
        marked = hostmesh.mark_fraction(-np.linalg.norm(cen, axis=1), frac)
        rg.refine(marked)
        cells, _ = rg.conforming()
    return rg.mesh("cube_corner_refined")


def config(i: int, L: Optional[int] = None) -> Workload:
    if i == 1:
        return Workload("unit_square_sine", meshes.unit_square_2tri(), L or 5, "redblack",
                        problems.sine2d_f, problems.zero, problems.sine2d_u)
    if i == 2:
        return Workload("lshape_corner", hostmesh.lshape_corner_refined(6), L or 9, "multicolour",
                        problems.zero, problems.lshape_u, problems.lshape_u)
    if i == 3:
        amp = problems.fourier_amplitudes(0)
        return Workload("cube_smooth_kappa", meshes.kuhn_cube(1), L or 7, "redblack",
                        lambda X: problems.fourier3d(X, amp), problems.zero, None,
                        coefficient="p1", kappa_nodal=problems.kappa_smooth3d)
    if i == 4:
        return Workload("cube_corner_singularity", _corner_refined_cube(), L or 5, "multicolour",
                        problems.corner3d_f, problems.corner3d_u, problems.corner3d_u)
    if i == 5:
        amp = problems.fourier_amplitudes(5)
        m = meshes.kuhn_cube(4)
        return Workload("cube_adjoint", m, L or 6, "redblack",
                        lambda X: problems.fourier3d(X, amp), problems.zero, None,
                        kappa_cell=problems.kappa_cells_uniform(55, m.n_cells),
                        goal_weight=problems.gaussian3d)
    if i == 6:
        amp = problems.fourier_amplitudes(0)
        return Workload("cube_uniform", meshes.kuhn_cube(1), L or 8, "redblack",
                        lambda X: problems.fourier3d(X, amp), problems.zero, None)
    raise ValueError(i)
