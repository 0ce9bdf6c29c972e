"""The FMG-based error estimator (Section 4; procedure ErrorEstimate of Algorithm 4).

With l = L - j and w_k the stored prolongation of the FMG solution of level k (w_k lives on
level k+1):
    e~_l     = u_L - I_{l+1}^L w_l,        e~_{l-1} = u_L - I_l^L w_{l-1}
    ||v||^2  = v^T N_L v                     (N_L = M_L: discrete L2 norm, Section 4.4)
    theta~_l = ||e~_l|| / ||e~_{l-1}||       (estimated convergence factor)
    eta_j    = theta~_l^j ||e~_l||           (global estimate)
Local indicators (Section 4.3), ||.||_T the norm over the fine elements of macro T only:
    eta_T     = ||e~_{L-1}||_T                      (the unscaled variant the paper implements
                                                     for P1, used for every j)
    eta'_{j,T} = ||e~_l||_T                         (unscaled, general j)
    eta_{j,T}  = theta~_{l,T}^j ||e~_l||_T,  theta~_{l,T} = ||e~_l||_T / ||e~_{l-1}||_T
so sum_T eta_T^2 = ||e~_{L-1}||^2.  A scaled indicator with ||e~_{l-1}||_T = 0 is set to 0
(the paper does not treat that case).

Norms (remark on the choice of norm, Section 4.4): "l2" uses the consistent mass matrix,
"energy" the stiffness matrix with the problem's coefficient, "lumped" the diagonal matrix of
mass-matrix row sums, |t|/(d+1) at each vertex of an element t.

``quadrature_l2`` integrates (v)^2 of a P1 field by a collapsed-coordinate Gauss product rule,
an independent check of the mass-matrix form; ``quadrature_energy`` does the same for
int kappa |grad(u - v_h)|^2.
"""
from __future__ import annotations

import math

import numpy as np

from . import assemble


def prolongate_to(solver, v, from_level, to_level):
    for k in range(from_level, to_level):
        v = solver.sys[k].P @ v
    return v


NORMS = ("l2", "energy", "lumped")


def element_norm_matrices(solver, norm: str = "l2"):
    """(ne, d+1, d+1) element matrices N_t of the fine level for the chosen norm."""
    h = solver.h
    lv = h.levels[h.L]
    if norm == "l2":
        return assemble.element_mass(lv.X, lv.E)
    if norm == "energy":
        kn = None if solver.kappa_nodal is None else np.asarray(solver.kappa_nodal)[:lv.n]
        kt = assemble.kappa_per_element(lv, solver.kappa_cell, kn)
        return assemble.element_stiffness(lv.X, lv.E, kt)
    if norm == "lumped":
        d = h.d
        _, vol = assemble.element_geometry(lv.X, lv.E)
        return vol[:, None, None] / (d + 1) * np.eye(d + 1)[None]
    raise ValueError(f"unknown norm {norm!r}")


def per_macro_sq_norms(h, v, Ne=None):
    """sum over the fine elements t of each macro of v_t^T N_t v_t (N_t: element mass matrix
    unless other element matrices are given)."""
    lv = h.levels[h.L]
    if Ne is None:
        Ne = assemble.element_mass(lv.X, lv.E)
    vt = v[lv.E]
    q = np.einsum("ei,eij,ej->e", vt, Ne, vt)
    return np.bincount(lv.emacro, weights=q, minlength=h.coarse_cells.shape[0])


def error_estimate(solver, u_L, w, j: int = 1, norm: str = "l2"):
    h = solver.h
    L = h.L
    if not (0 < j < L):
        raise ValueError("need 0 < j < L")
    Ne = element_norm_matrices(solver, norm)
    l = L - j
    a = prolongate_to(solver, w[l], l + 1, L)          # I_{l+1}^L w_l
    b = prolongate_to(solver, w[l - 1], l, L)          # I_l^L w_{l-1}
    e_l = u_L - a
    e_lm1 = u_L - b
    T_l = per_macro_sq_norms(h, e_l, Ne)
    T_lm1 = per_macro_sq_norms(h, e_lm1, Ne)
    n_l = math.sqrt(T_l.sum())
    n_lm1 = math.sqrt(T_lm1.sum())
    theta = n_l / n_lm1
    eta_j = theta ** j * n_l
    if j == 1:
        T_L1 = T_l
    else:
        T_L1 = per_macro_sq_norms(h, u_L - w[L - 1], Ne)
    eta_T = np.sqrt(T_L1)
    eta_prime_jT = np.sqrt(T_l)
    den = np.sqrt(T_lm1)
    eta_jT = np.zeros_like(eta_prime_jT)
    nz = den > 0
    eta_jT[nz] = (eta_prime_jT[nz] / den[nz]) ** j * eta_prime_jT[nz]
    return dict(eta_T=eta_T, eta_j=eta_j, theta=theta, norm_e_l=n_l, norm_e_lm1=n_lm1,
                sq_l=T_l, sq_lm1=T_lm1, eta_jT=eta_jT, eta_prime_jT=eta_prime_jT, e_l=e_l, e_lm1=e_lm1)


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


def quadrature_energy(h, nodal, grad_exact=None, kappa_el=None, m: int = 4, per_macro: bool = False,
                      chunk: int = 200000):
    """sqrt(int kappa |grad u - grad v_h|^2) (grad_exact=None: int kappa |grad v_h|^2) for the
    P1 field v_h with the given nodal values on the fine level.  The element gradient of v_h is
    the solution g of (x_a - x_0) . g = v_a - v_0, a = 1..d; grad u is integrated with the
    collapsed Gauss rule of m^d points.  kappa_el: per fine element (None = 1).  With
    per_macro, returns the squared integrals per macro instead."""
    lv = h.levels[h.L]
    d = h.d
    ref, W = _collapsed_rule(d, m)
    lam = np.concatenate([1.0 - ref.sum(axis=1, keepdims=True), ref], axis=1)
    nmac = h.coarse_cells.shape[0]
    acc = np.zeros(nmac)
    for s in range(0, lv.E.shape[0], chunk):
        E = lv.E[s:s + chunk]
        P = lv.X[E]
        Dx = P[:, 1:, :] - P[:, :1, :]                        # rows x_a - x_0
        dv = nodal[E][:, 1:] - nodal[E][:, :1]
        g = np.linalg.solve(Dx, dv[..., None])[..., 0]        # (ne, d)
        det = np.abs(np.linalg.det(Dx))
        if grad_exact is None:
            val = (g * g).sum(axis=1) * det / math.factorial(d)
        else:
            pts = np.einsum("qa,ead->eqd", lam, P).reshape(-1, d)
            ge = grad_exact(pts).reshape(E.shape[0], -1, d)   # (ne, q, d)
            diff = ge - g[:, None, :]
            val = ((diff * diff).sum(axis=2) * W[None, :]).sum(axis=1) * det
        if kappa_el is not None:
            val = val * np.asarray(kappa_el)[s:s + chunk]
        acc += np.bincount(lv.emacro[s:s + chunk], weights=val, minlength=nmac)
    return acc if per_macro else math.sqrt(float(acc.sum()))
