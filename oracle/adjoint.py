"""Gradient of a goal functional of the converged discrete solution.

The paper only mentions goal-oriented (semi-)norms (remark on norm choices in Section 4.4);
the reading here: for J(u_h) with u_h = A^{-1} b, b = M f on inner rows and u_h = g on the
Dirichlet boundary,
    adjoint:   A_II lambda_I = (dJ/du)_I,   lambda = 0 on Dirichlet nodes
    dJ/df    = M lambda                (f enters only through b = M f)
    dJ/dk_e  = -lambda^T A_e u_h       (A_e: unit-coefficient stiffness of macro e's elements)
This differentiates the exact discrete solution, not the truncated iteration.
"""
from __future__ import annotations

import numpy as np

from . import assemble


def gradient(solver, f_fine, g_fine, dJdu):
    h = solver.h
    L = h.L
    s = solver.sys[L]
    b = s.M @ np.asarray(f_fine)
    u = solver.direct(L, b, g_fine)
    lam = solver.direct(L, np.asarray(dJdu, dtype=np.float64), np.zeros(s.N))
    dJdf = s.M @ lam
    lv = h.levels[L]
    Ke = assemble.element_stiffness(lv.X, lv.E, None)
    q = np.einsum("ei,eij,ej->e", lam[lv.E], Ke, u[lv.E])
    dJdk = -np.bincount(lv.emacro, weights=q, minlength=h.coarse_cells.shape[0])
    return dict(u=u, lam=lam, dJdf=dJdf, dJdkappa=dJdk)
