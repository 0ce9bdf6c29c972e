"""kl-refinement driven by the library (Section 3, Algorithm "kl-Refinement").

For k = 0, ..., K-1: refine every macro of the current coarse mesh T_0^k uniformly L times (the
HHG hierarchy of ``hhg_setup``), solve on T_L^k by FMG with extra V-cycles on level L, compute
one value per macro, mark the fraction of macros with the largest values and refine T_0^k by
red-green refinement (greens reverted between steps).  A last solve on T_L^K ends the loop.

Refinement criterion (one value per macro T):
* ``"error"``: the local error ||I_L u - u_L||_T against the nodal interpolant of a known
  solution u, the criterion of the convergence studies (Sections 5.1 and 5.2 drive the
  refinement by the actual local L2 errors so that the estimator does not influence them);
* ``"estimate"``: the indicator eta_T = ||u_L - w_{L-1}||_T of Section 4.4.

Every fine-grid step (setup tables, solve, local norms, estimate) runs in the HIP library; the
macro mesh is small, so marking and red-green refinement run serially on the host, as in the
paper.  Errors are discrete L2 norms (mass matrix of level L).  The data callables f, g and u
receive the level-L DoF coordinates as a device tensor and return nodal values (numpy results
are copied to the device).

Warm start (``warm=True``, the solution transfer the conclusion of the paper lists as future
work): from the second step on, the solution on T_L^k is evaluated at the DoFs of T_L^(k+1)
(``hhg_transfer``) and V-cycles run from there (``hhg_cycle_solve``) instead of an FMG solve.
No FMG levels exist then, so these steps carry neither eta_T nor a level-0 error, and the
criterion must be ``"error"``.

Mesh-quality metric (Section 5.1, equation of the error ratio): with hbar = (|Omega| / #T)^(1/d)
the mean mesh width of T_L^k, Hbar that of T_0^0, e_hbar the error on T_L^k and e_Hbar the error
of the solution on T_0^0,
    rho = Hbar^2 ||e_hbar|| / (hbar^2 ||e_Hbar||),
which stays near a constant for a quasi-optimal sequence (1 marks the O(hbar^2) line through
the coarse-grid error).  e_Hbar is taken from the level-0 FMG solution of the first step,
measured against the level-L nodal interpolant of u (``hhg_macro_norms`` with level 0).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from workloads.meshes import CoarseMesh

from . import mesh as hostmesh


@dataclass
class KStep:
    k: int
    mesh: CoarseMesh
    n_dofs: int
    hbar: float
    err: Optional[float]                  # ||I_L u - u_L|| (None without an exact solution)
    err_level0: Optional[float]           # error of the level-0 FMG solution of this step
    eta_1: float
    theta: float
    local: np.ndarray                     # the per-macro criterion values
    marked: Optional[np.ndarray]          # macros marked for red refinement (None: last solve)
    vcycles: int
    t_setup: float                        # seconds, host clock around each phase
    t_solve: float
    t_local: float
    t_refine: float
    extra: dict = field(default_factory=dict)

    @property
    def n_macros(self) -> int:
        return self.mesh.n_cells


def domain_measure(mesh: CoarseMesh) -> float:
    X = np.asarray(mesh.coords, dtype=np.float64)
    P = X[np.asarray(mesh.cells)]
    J = P[:, 1:, :] - P[:, :1, :]
    return float(np.abs(np.linalg.det(J)).sum()) / math.factorial(mesh.dim)


def mean_width(mesh: CoarseMesh, level: int, measure: Optional[float] = None) -> float:
    """hbar = (|Omega| / #T)^(1/d) of T_level: every macro holds 2^(d level) fine elements."""
    d = mesh.dim
    n = mesh.n_cells * (2 ** (d * level))
    return ((domain_measure(mesh) if measure is None else measure) / n) ** (1.0 / d)


def error_ratio(steps: List[KStep]) -> List[float]:
    """rho of every step relative to the coarse grid T_0^0 of the first step."""
    if not steps or steps[0].err_level0 is None:
        raise ValueError("needs the error of the level-0 solution of the first step")
    m0 = steps[0].mesh
    H = mean_width(m0, 0)
    eH = steps[0].err_level0
    return [(H * H * s.err) / (s.hbar * s.hbar * eH) for s in steps]


def effectivity(steps: List[KStep], j: int) -> List[float]:
    """gamma_j = eta_j / ||e_L|| per step (Section 5.3); needs ``estimate_js`` to hold j."""
    return [s.extra["eta"][j] / s.err for s in steps]


def worst_effectivity(steps: List[KStep], j: int):
    """(k, gamma_j) of the step whose |log gamma_j| is largest: the worst case of Section 5.3."""
    g = effectivity(steps, j)
    k = max(range(len(g)), key=lambda i: abs(math.log(g[i])))
    return steps[k].k, g[k]


def _solve_until_stable(hh, fd, gd, ud, L, nu, precision, rtol, max_iter, tighten):
    """FMG solves, each from scratch, with the tolerance lowered until the error is stable.
    Returns (stats of the last solve, per-macro squared errors, number of solves, u_L)."""
    from ._lib import HHG_ENOTCONV, HHGError
    prev = sq = st = u = None
    n = 0
    for t in range(tighten + 1):
        try:
            u_t, st_t = hh.fmg_solve(fd, gd, nu=nu, precision=precision, rtol=rtol * 100.0 ** (-t), max_iter=max_iter)
        except HHGError as e:
            if e.status != HHG_ENOTCONV or st is None:
                raise
            # the tighter tolerance is below what float64 reaches: repeat the last solve
            u, st = hh.fmg_solve(fd, gd, nu=nu, precision=precision, rtol=rtol * 100.0 ** (1 - t), max_iter=max_iter)
            n += 1
            if ud is not None:
                sq = hh.macro_norms(ud, L)
            break
        n += 1
        u, st = u_t, st_t
        if ud is None:
            break
        sq = hh.macro_norms(ud, L)
        err = f"{math.sqrt(float(sq.sum())):.1e}"
        if err == prev:
            break
        prev = err
    return st, sq, n, u


def _cycles_until_stable(hh, fd, gd, u, ud, L, precision, rtol, max_iter, tighten):
    """V-cycles from the iterate u, continued with the tolerance lowered until the error is
    stable.  Returns (stats with the V-cycles of all rounds, squared errors, rounds, u_L)."""
    from ._lib import HHG_ENOTCONV, HHGError, SolveStats
    prev = sq = st = None
    n = cycles = 0
    for t in range(tighten + 1):
        try:
            u_t, st_t = hh.cycle_solve(fd, gd, u, precision=precision, rtol=rtol * 100.0 ** (-t), max_iter=max_iter)
        except HHGError as e:
            if e.status != HHG_ENOTCONV or st is None:
                raise
            break                      # the last iterate and its errors stand
        n += 1
        cycles += st_t.vcycles
        u, st = u_t, st_t
        if ud is None:
            break
        sq = hh.macro_norms(ud, L)
        err = f"{math.sqrt(float(sq.sum())):.1e}"
        if err == prev:
            break
        prev = err
    return SolveStats(cycles, st.ir_steps, st.final_rel_residual, st.ms_total), sq, n, u


def _nodal(fn, X, device):
    import torch
    return torch.as_tensor(fn(X), dtype=torch.float64, device=device).contiguous()


def kl_refine(coarse: CoarseMesh, L: int, K: int, f: Callable, g: Callable,
              u_exact: Optional[Callable] = None, criterion: str = "error", fraction: float = 0.1,
              smoother: str = "multicolour", nu: int = 2, rtol: float = 1e-10, max_iter: int = 100,
              precision: str = "fp64", device: str = "cuda:0", tighten: int = 3, warm: bool = False,
              estimate_js: Sequence[int] = (),
              callback: Optional[Callable[[KStep], None]] = None) -> List[KStep]:
    """Run K kl-steps and the final solve; returns one record per solved mesh (K + 1).

    Each solve is FMG plus extra V-cycles to the relative residual ``rtol``; with a known
    solution it is repeated with the tolerance lowered 100-fold (at most ``tighten`` times)
    until the first two significant digits of the error no longer change, the stopping rule
    of the experiments in Section 5.  For every j in ``estimate_js`` (1 <= j < L) each FMG step
    also records the global estimate eta_j in ``extra["eta"][j]``."""
    import torch
    from ._lib import HHG, HHG_FLAG_NO_DENSE_COARSE

    if criterion not in ("error", "estimate"):
        raise ValueError("criterion is 'error' or 'estimate'")
    if criterion == "error" and u_exact is None:
        raise ValueError("the 'error' criterion needs u_exact")
    if criterion == "estimate" and L < 2:
        raise ValueError("the estimate needs L >= 2")
    for j in estimate_js:
        if not 1 <= j < L:
            raise ValueError(f"eta_{j} needs 1 <= j < L = {L}")
    if warm and criterion != "error":
        raise ValueError("warm-started steps have no FMG levels, hence no estimate: use criterion 'error'")
    if coarse.dim == 2:
        rg = hostmesh.RedGreen2D(coarse)
    else:
        rg = hostmesh.RedGreen3D(coarse)
    measure = domain_measure(coarse)
    steps: List[KStep] = []
    prev = None                                    # (context, u_L) of the last step, for the warm start
    for k in range(K + 1):
        m = rg.mesh(f"{coarse.name}_k{k}")          # macro order = conforming-cell order
        t0 = time.perf_counter()
        # one context per mesh, solved once (or a few warm rounds): the dense map of the coarse
        # cycle would cost about one probe cycle per coarse DoF and never pay off here
        hh = HHG(m.coords, m.cells, L, smoother=smoother, device=device, flags=HHG_FLAG_NO_DENSE_COARSE)
        X = hh.dof_coords()
        fd, gd = _nodal(f, X, hh.device), _nodal(g, X, hh.device)
        ud = None if u_exact is None else _nodal(u_exact, X, hh.device)
        del X
        torch.cuda.synchronize(hh.device)
        t1 = time.perf_counter()
        t_transfer = 0.0
        if warm and prev is not None:
            u0 = hh.transfer_from(prev[0], prev[1])
            torch.cuda.synchronize(hh.device)
            t_transfer = time.perf_counter() - t1
            prev[0].close()
            prev = None
            st, sq, n_solves, u = _cycles_until_stable(hh, fd, gd, u0, ud, L, precision, rtol, max_iter, tighten)
        else:
            st, sq, n_solves, u = _solve_until_stable(hh, fd, gd, ud, L, nu, precision, rtol, max_iter, tighten)
        torch.cuda.synchronize(hh.device)
        t2 = time.perf_counter()
        fmg_levels = not (warm and k > 0)
        est = hh.estimate(1) if L >= 2 and fmg_levels else dict(eta_j=math.nan, theta=math.nan, eta_T=None)
        eta = {}
        if fmg_levels:
            for j in estimate_js:
                eta[j] = est["eta_j"] if j == 1 else hh.estimate(j)["eta_j"]
        err = err0 = None
        if ud is not None:
            err = math.sqrt(float(sq.sum()))
            if fmg_levels:
                err0 = math.sqrt(float(hh.macro_norms(ud, 0).sum()))
        local = np.sqrt(sq) if criterion == "error" else est["eta_T"]
        t3 = time.perf_counter()
        marked = None
        if k < K:
            marked = hostmesh.mark_fraction(local, fraction)
            rg.refine(marked)
        t4 = time.perf_counter()
        s = KStep(k, m, hh.num_dofs(), mean_width(m, L, measure), err, err0, est["eta_j"], est["theta"], local,
                  marked, st.vcycles, t1 - t0, t2 - t1, t3 - t2, t4 - t3,
                  dict(solves=n_solves, final_rel_residual=st.final_rel_residual, transfer_s=t_transfer, eta=eta))
        steps.append(s)
        if callback is not None:
            callback(s)
        del fd, gd, ud
        if warm and k < K:
            prev = (hh, u)
        else:
            hh.close()
        del hh, u
    return steps
