"""The FMG-based error estimator (Section 4; procedure ErrorEstimate of Algorithm 4).

With l = L - j and w_k the stored prolongation of the FMG solution of level k (w_k lives on
level k+1):
    e~_l     = u_L - I_{l+1}^L w_l,        e~_{l-1} = u_L - I_l^L w_{l-1}
    ||v||^2  = v^T M_L v                     (discrete L2 norm, Section 4.5)
    theta~_l = ||e~_l|| / ||e~_{l-1}||       (estimated convergence factor)
    eta_j    = theta~_l^j ||e~_l||           (global estimate)
Local indicator (the unscaled variant the paper implements for P1):
    eta_T = ||e~_{L-1}||_T,  the L2 norm over the fine elements of macro T only,
so sum_T eta_T^2 = ||e~_{L-1}||^2.  Also returns the scaled local variant
eta_{j,T} = theta~_{l,T}^j ||e~_l||_T.

``quadrature_l2`` integrates (v)^2 of a P1 field by a collapsed-coordinate Gauss product rule,
an independent check of the mass-matrix form.
"""
from __future__ import annotations

import math

import numpy as np

from . import assemble


def prolongate_to(solver, v, from_level, to_level):
    for k in range(from_level, to_level):
        v = solver.sys[k].P @ v
    return v


def per_macro_sq_norms(h, v):
    """sum over the fine elements t of each macro of v_t^T M_t v_t."""
    lv = h.levels[h.L]
    Me = assemble.element_mass(lv.X, lv.E)
    vt = v[lv.E]
    q = np.einsum("ei,eij,ej->e", vt, Me, vt)
    return np.bincount(lv.emacro, weights=q, minlength=h.coarse_cells.shape[0])


def error_estimate(solver, u_L, w, j: int = 1):
    h = solver.h
    L = h.L
    if not (0 < j < L):
        raise ValueError("need 0 < j < L")
    l = L - j
    a = prolongate_to(solver, w[l], l + 1, L)          # I_{l+1}^L w_l
    b = prolongate_to(solver, w[l - 1], l, L)          # I_l^L w_{l-1}
    e_l = u_L - a
    e_lm1 = u_L - b
    T_l = per_macro_sq_norms(h, e_l)
    T_lm1 = per_macro_sq_norms(h, e_lm1)
    n_l = math.sqrt(T_l.sum())
    n_lm1 = math.sqrt(T_lm1.sum())
    theta = n_l / n_lm1
    eta_j = theta ** j * n_l
    if j == 1:
        T_L1 = T_l
    else:
        T_L1 = per_macro_sq_norms(h, u_L - w[L - 1])
    eta_T = np.sqrt(T_L1)
    with np.errstate(divide="ignore", invalid="ignore"):
        theta_T = np.sqrt(T_l) / np.sqrt(T_lm1)
    eta_jT = theta_T ** j * np.sqrt(T_l)
    return dict(eta_T=eta_T, eta_j=eta_j, theta=theta, norm_e_l=n_l, norm_e_lm1=n_lm1,
                sq_l=T_l, sq_lm1=T_lm1, eta_jT=eta_jT, e_l=e_l, e_lm1=e_lm1)


def effectivity_bounds(theta: float, eps: float, j: int):
    """Closed-form constants C1, C2 of the theorem on eta_j bounds."""
    te = (1.0 + eps) * theta
    C1 = (1.0 + eps) ** (-j) * (1.0 - te ** j) ** (j + 1) / (1.0 + te ** (j + 1)) ** j
    C2 = (1.0 + eps) ** j * (1.0 + te ** j) ** (j + 1) / (1.0 - te ** (j + 1)) ** j
    return C1, C2


# --- quadrature ------------------------------------------------------------------------------
def _collapsed_rule(d: int, m: int):
    """Points (barycentric-free, reference simplex) and weights of the conical product rule
    built from m-point Gauss-Legendre rules mapped to [0, 1] (Duffy / Stroud construction)."""
    x, wgt = np.polynomial.legendre.leggauss(m)
    x = 0.5 * (x + 1.0)
    wgt = 0.5 * wgt
    if d == 2:
        s, t = np.meshgrid(x, x, indexing="ij")
        ws, wt = np.meshgrid(wgt, wgt, indexing="ij")
        px = s
        py = t * (1.0 - s)
        W = ws * wt * (1.0 - s)
        return np.stack([px.ravel(), py.ravel()], 1), W.ravel()
    s, t, r = np.meshgrid(x, x, x, indexing="ij")
    ws, wt, wr = np.meshgrid(wgt, wgt, wgt, indexing="ij")
    px = s
    py = t * (1.0 - s)
    pz = r * (1.0 - s) * (1.0 - t)
    W = ws * wt * wr * (1.0 - s) ** 2 * (1.0 - t)
    return np.stack([px.ravel(), py.ravel(), pz.ravel()], 1), W.ravel()


def quadrature_l2(h, nodal, exact=None, m: int = 4, level=None, chunk: int = 200000):
    """sqrt(int (exact - v_h)^2) for the P1 field with the given nodal values (exact=None
    integrates v_h^2), element by element with a collapsed Gauss rule of m^d points."""
    lv = h.levels[h.L if level is None else level]
    d = h.d
    ref, W = _collapsed_rule(d, m)
    lam = np.concatenate([1.0 - ref.sum(axis=1, keepdims=True), ref], axis=1)   # (q, d+1)
    total = 0.0
    for s in range(0, lv.E.shape[0], chunk):
        E = lv.E[s:s + chunk]
        P = lv.X[E]                                       # (ne, d+1, d)
        J = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))
        det = np.abs(np.linalg.det(J))
        vh = lam @ nodal[E].T                              # (q, ne)
        if exact is not None:
            pts = np.einsum("qa,ead->eqd", lam, P).reshape(-1, d)
            ue = exact(pts).reshape(E.shape[0], -1).T
            diff = ue - vh
        else:
            diff = vh
        total += float(np.sum((W[:, None] * diff * diff) * det[None, :]))
    return math.sqrt(total)


def discrete_l2_error(solver, u_h, u_exact_nodal):
    e = u_exact_nodal - u_h
    return math.sqrt(float(e @ (solver.sys[solver.L].M @ e)))
