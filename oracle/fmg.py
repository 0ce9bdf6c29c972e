"""Textbook full multigrid (Algorithm 4, procedure FMG) on assembled level matrices.

Structure (float64 throughout):
* level 0: exact solve of the inner block by dense Cholesky.  The paper uses CG to a 1e-9
  residual there; an exact solve is the reading taken so that two implementations agree to
  round-off.  "nu V-cycles on level 0" therefore reduce to one exact solve.
* V-cycle(l): nu1 forward Gauss-Seidel colour sweeps (or damped Jacobi), residual
  r = b - A u (zero on Dirichlet rows), restriction r_c = P^T r (zero on coarse Dirichlet
  rows), recursive correction solve from zero, u += P e_c on inner nodes, nu2 sweeps.
* FMG: for l = 1..L, w_{l-1} <- P u_{l-1} (the unmodified prolongation is what the estimator
  compares against), u_l <- w_{l-1} with the nodal Dirichlet data g_l written on boundary
  nodes, then nu V-cycles.  Writing g_l after prolongation is not spelled out by Algorithm 4;
  it changes nothing when g is piecewise linear on the boundary.
* optional extra V-cycles on level L (Section 5 runs extra cycles after FMG until the error
  stops changing; the coarse solutions w are not touched by them).
* reduced-precision cycle (the float32-refined form): the residual r = b - A u is formed in
  float64 and rounded to the working precision, a V-cycle on the correction equation A e = r
  runs from e = 0 entirely in that precision (operator, smoother, transfers rounded to it),
  except level 0, whose exact solve is float64 and rounded afterwards; then u += e in
  float64.  u, w, the FMG prolongation and the level-0 solve of the FMG pass stay float64,
  because the estimator differences u_L - w_l are of the size of the algebraic error the
  remark on algebraic errors in Section 4.2 warns about.  With float64 as the working
  precision the cycle is the correction form of the float64 V-cycle (equal up to round-off,
  multigrid being affine).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assemble, colour


class LevelSystem:
    def __init__(self, h, l, kappa_cell, kappa_nodal_fine, smoother):
        lv = h.levels[l]
        self.l = l
        self.N = lv.n
        kn = None if kappa_nodal_fine is None else np.asarray(kappa_nodal_fine)[:lv.n]
        self.A = assemble.stiffness(lv, kappa_cell, kn)
        self.M = assemble.mass(lv)
        self.bnd = lv.boundary.copy()
        self.inner = np.nonzero(~self.bnd)[0]
        self.diag = self.A.diagonal()
        if smoother == "redblack":
            self.col = colour.red_black(h, l)
        elif smoother == "multicolour":
            self.col = colour.multicolour(h, l)
        else:
            self.col = np.where(self.bnd, -1, 0)
        self.classes = colour.classes(self.col)
        self.rows = [self.A[c] for c in self.classes]
        self.P = assemble.prolongation(h, l) if l < h.L else None
        self._lowp = {}

    def lowp(self, dtype):
        """Operator, smoother rows, diagonal and prolongation rounded to ``dtype``."""
        dt = np.dtype(dtype)
        if dt not in self._lowp:
            self._lowp[dt] = dict(
                A=self.A.astype(dt), rows=[R.astype(dt) for R in self.rows], diag=self.diag.astype(dt),
                P=None if self.P is None else self.P.astype(dt), PT=None if self.P is None else self.P.T.tocsr().astype(dt))
        return self._lowp[dt]


class FMGSolver:
    def __init__(self, h, kappa_cell=None, kappa_nodal=None, smoother="redblack",
                 omega=2.0 / 3.0, nu1=2, nu2=2):
        self.h = h
        self.L = h.L
        self.kappa_cell = kappa_cell
        self.kappa_nodal = kappa_nodal
        self.smoother = smoother
        self.omega = omega
        self.nu1, self.nu2 = nu1, nu2
        self.sys = [LevelSystem(h, l, kappa_cell, kappa_nodal, smoother) for l in range(h.L + 1)]
        s0 = self.sys[0]
        I = s0.inner
        self.coarse_inner = I
        if I.size:
            A_II = s0.A[I][:, I].toarray()
            self.coarse_factor = sla.cho_factor(A_II)
        else:
            self.coarse_factor = None

    # --- building blocks -------------------------------------------------------------------
    def smooth(self, l, u, b, sweeps):
        s = self.sys[l]
        for _ in range(sweeps):
            if self.smoother == "jacobi":
                r = b - s.A @ u
                u[s.inner] += self.omega * r[s.inner] / s.diag[s.inner]
            else:
                for idx, R in zip(s.classes, s.rows):
                    u[idx] += (b[idx] - R @ u) / s.diag[idx]

    def residual(self, l, u, b):
        s = self.sys[l]
        r = b - s.A @ u
        r[s.bnd] = 0.0
        return r

    def coarse_solve(self, u, b):
        s0 = self.sys[0]
        I = s0.inner
        if I.size == 0:
            return
        rhs = b[I] - (s0.A[I] @ np.where(s0.bnd, u, 0.0))
        u[I] = sla.cho_solve(self.coarse_factor, rhs)

    def vcycle(self, l, u, b):
        if l == 0:
            self.coarse_solve(u, b)
            return
        s, sc = self.sys[l], self.sys[l - 1]
        self.smooth(l, u, b, self.nu1)
        r = self.residual(l, u, b)
        rc = sc.P.T @ r
        rc[sc.bnd] = 0.0
        ec = np.zeros(sc.N)
        self.vcycle(l - 1, ec, rc)
        corr = sc.P @ ec
        u[s.inner] += corr[s.inner]
        self.smooth(l, u, b, self.nu2)

    # --- reduced-precision correction cycle (float32-refined form) ---------------------------
    def smooth_lowp(self, l, e, r, sweeps, dtype):
        s = self.sys[l]
        q = s.lowp(dtype)
        om = np.asarray(self.omega, dtype=dtype)
        for _ in range(sweeps):
            if self.smoother == "jacobi":
                res = r - q["A"] @ e
                e[s.inner] += om * res[s.inner] / q["diag"][s.inner]
            else:
                for idx, R in zip(s.classes, q["rows"]):
                    e[idx] += (r[idx] - R @ e) / q["diag"][idx]

    def vcycle_lowp(self, l, e, r, dtype):
        """V(nu1, nu2) cycle for A_l e = r from e = 0 with every vector and operator in
        ``dtype``; level 0 is the float64 exact solve of the rounded right-hand side, rounded
        back."""
        dt = np.dtype(dtype)
        if l == 0:
            # reached from the cycle above with e = 0 (zero on Dirichlet nodes as well)
            I = self.sys[0].inner
            if I.size:
                e[I] = sla.cho_solve(self.coarse_factor, r[I].astype(np.float64)).astype(dt)
            return
        s, sc = self.sys[l], self.sys[l - 1]
        q, qc = s.lowp(dt), sc.lowp(dt)
        self.smooth_lowp(l, e, r, self.nu1, dt)
        res = r - q["A"] @ e
        res[s.bnd] = 0
        rc = qc["PT"] @ res
        rc[sc.bnd] = 0
        ec = np.zeros(sc.N, dtype=dt)
        self.vcycle_lowp(l - 1, ec, rc, dt)
        corr = qc["P"] @ ec
        e[s.inner] += corr[s.inner]
        self.smooth_lowp(l, e, r, self.nu2, dt)

    def refined_cycle(self, l, u, b, dtype=np.float32):
        """One step of the refinement loop: float64 residual rounded to ``dtype``, a ``dtype``
        V-cycle on the correction from zero, float64 update u += e."""
        dt = np.dtype(dtype)
        r = self.residual(l, u, b).astype(dt)
        e = np.zeros(self.sys[l].N, dtype=dt)
        self.vcycle_lowp(l, e, r, dt)
        u += e.astype(np.float64)

    def _cycle(self, l, u, b, precision):
        if precision == "fp64":
            self.vcycle(l, u, b)
        elif precision == "fp32_refined":
            self.refined_cycle(l, u, b, np.float32)
        else:
            raise ValueError(f"unknown precision {precision!r}")

    # --- right-hand sides --------------------------------------------------------------------
    def rhs_levels(self, f_fine):
        """b_l = M_l f_l with f_l the nodal values on level l (nested numbering: the first N_l
        fine values)."""
        return [s.M @ np.asarray(f_fine)[:s.N] for s in self.sys]

    def rhs_restricted(self, b_fine):
        """Right-hand sides for a system given only on the fine level (adjoint): coarse levels
        receive P^T-restrictions of the fine one."""
        bs = [None] * (self.L + 1)
        bs[self.L] = np.asarray(b_fine, dtype=np.float64).copy()
        for l in range(self.L, 0, -1):
            r = bs[l].copy()
            r[self.sys[l].bnd] = 0.0
            bs[l - 1] = self.sys[l - 1].P.T @ r
        return bs

    # --- FMG ------------------------------------------------------------------------------
    def fmg(self, b_levels, g_fine, nu=1, precision="fp64"):
        """precision "fp32_refined": every V-cycle of the pass is a refined_cycle in float32;
        the level-0 solve, the prolongations, u and w stay float64."""
        g_fine = np.asarray(g_fine)
        s0 = self.sys[0]
        u = np.where(s0.bnd, g_fine[:s0.N], 0.0)
        self.coarse_solve(u, b_levels[0])
        w = [None] * self.L
        for l in range(1, self.L + 1):
            s = self.sys[l]
            v = self.sys[l - 1].P @ u
            w[l - 1] = v.copy()
            u = v
            u[s.bnd] = g_fine[:s.N][s.bnd]
            for _ in range(nu):
                self._cycle(l, u, b_levels[l], precision)
        return u, w

    def ref_residual(self, b, g_fine):
        sL = self.sys[self.L]
        u0 = np.where(sL.bnd, np.asarray(g_fine)[:sL.N], 0.0)
        return float(np.linalg.norm(self.residual(self.L, u0, b)))

    def extra_cycles(self, u, b, g_fine, rtol=0.0, max_iter=0, precision="fp64"):
        """Further V-cycles on level L until ||r|| <= rtol * ||r(u = g on boundary, 0 inside)||
        (precision "fp32_refined": refinement steps with a float32 cycle)."""
        r0 = self.ref_residual(b, g_fine)
        it = 0
        rel = float(np.linalg.norm(self.residual(self.L, u, b))) / r0 if r0 > 0 else 0.0
        while it < max_iter and rel > rtol:
            self._cycle(self.L, u, b, precision)
            it += 1
            rel = float(np.linalg.norm(self.residual(self.L, u, b))) / r0 if r0 > 0 else 0.0
        return it, rel

    # --- direct solve ----------------------------------------------------------------------
    def direct(self, l, b, g_fine):
        s = self.sys[l]
        I = s.inner
        u = np.where(s.bnd, np.asarray(g_fine)[:s.N], 0.0)
        rhs = b[I] - s.A[I] @ u
        u[I] = spla.spsolve(s.A[I][:, I].tocsc(), rhs)
        return u


def solve(h, f_fine, g_fine, kappa_cell=None, kappa_nodal=None, smoother="redblack",
          nu=1, nu1=2, nu2=2, omega=2.0 / 3.0, rtol=0.0, max_iter=0):
    """Convenience driver: FMG followed by optional extra cycles.  Returns (u_L, w, solver)."""
    S = FMGSolver(h, kappa_cell, kappa_nodal, smoother, omega, nu1, nu2)
    b = S.rhs_levels(f_fine)
    u, w = S.fmg(b, g_fine, nu)
    if max_iter:
        S.extra_cycles(u, b[h.L], g_fine, rtol, max_iter)
    return u, w, S
