"""Element-by-element assembly of the level matrices (Section 4.4, the per-level linear
system A_l u_l = b_l, and Section 5, the Poisson form a(u,v) = int grad v . grad u,
b(v) = int v f).

* Stiffness: A = sum_t kappa_t |t| grad(lambda_i) . grad(lambda_j) (P1 hat functions).
  kappa_t is the macro element's constant, or, for a nodal (P1) coefficient, the mean of the
  nodal values at the element's vertices (the exact element integral of the P1 interpolant).
* Mass: M = sum_t |t| (1 + delta_ij) / ((d+1)(d+2)), the consistent P1 mass matrix.
* Load vector on every level: b_l = M_l f_l with f_l the nodal interpolant of f.
* Prolongation P_l : level l -> level l+1, injection at old nodes and 1/2, 1/2 at edge
  midpoints (the refinement relation recorded by ``refine``); restriction is P_l^T.
Everything is float64; duplicates are summed by scipy when converting COO to CSR.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def element_geometry(X: np.ndarray, E: np.ndarray):
    """Return (grads, vol): grads (ne, d+1, d) gradients of the barycentric functions,
    vol (ne,) element measures."""
    d = X.shape[1]
    P = X[E]                                   # (ne, d+1, d)
    J = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))   # columns y_k - y_0: (ne, d, d)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                    # rows are grad(lambda_k), k = 1..d
    g = np.empty((E.shape[0], d + 1, d))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    vol = np.abs(det) / math.factorial(d)
    return g, vol


def element_stiffness(X, E, kappa_el=None):
    g, vol = element_geometry(X, E)
    K = np.einsum("eid,ejd->eij", g, g) * vol[:, None, None]
    if kappa_el is not None:
        K = K * np.asarray(kappa_el)[:, None, None]
    return K


def element_mass(X, E):
    d = X.shape[1]
    _, vol = element_geometry(X, E)
    base = (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    return vol[:, None, None] * base[None]


def _scatter(E, Ke, N):
    d1 = E.shape[1]
    rows = np.repeat(E, d1, axis=1).ravel()
    cols = np.tile(E, (1, d1)).ravel()
    return sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(N, N)).tocsr()


def kappa_per_element(lv, kappa_cell=None, kappa_nodal=None):
    """kappa_t for every element of a level: macro constant, or mean of nodal values."""
    if kappa_nodal is not None:
        return np.asarray(kappa_nodal)[lv.E].mean(axis=1)
    if kappa_cell is not None:
        return np.asarray(kappa_cell)[lv.emacro]
    return None


def stiffness(lv, kappa_cell=None, kappa_nodal=None):
    kt = kappa_per_element(lv, kappa_cell, kappa_nodal)
    return _scatter(lv.E, element_stiffness(lv.X, lv.E, kt), lv.n)


def mass(lv):
    return _scatter(lv.E, element_mass(lv.X, lv.E), lv.n)


def prolongation(h, l: int):
    """P_l : R^{N_l} -> R^{N_{l+1}}."""
    lv = h.levels[l]
    Nc, Nf = h.levels[l].n, h.levels[l + 1].n
    par = lv.parents
    newi = np.arange(Nc, Nf)
    rows = np.concatenate([np.arange(Nc), newi, newi])
    cols = np.concatenate([np.arange(Nc), par[:, 0], par[:, 1]])
    vals = np.concatenate([np.ones(Nc), np.full(Nf - Nc, 0.5), np.full(Nf - Nc, 0.5)])
    return sp.coo_matrix((vals, (rows, cols)), shape=(Nf, Nc)).tocsr()


def macro_stiffness_parts(lv, n_macro: int):
    """Per-macro unit-coefficient stiffness matrices A_e (sum over the macro's own elements),
    returned as element arrays so callers can form lambda^T A_e u by a bincount."""
    return element_stiffness(lv.X, lv.E, None)
