"""Transfer of a P1 function from the fine level of one macro mesh to the nodes of another
mesh of the same domain: the solution transfer from T_L^k to T_L^(k+1) that the conclusion
(Section 6) lists as missing for kl-refinement.

The value at a point p is the old P1 function at p: find an element t of the old fine mesh
that contains p (all barycentric coordinates of p in t >= -tol) and return
sum_a lambda_a(p) u(vertex_a of t).  Where elements share p (on an edge or at a vertex) every
choice gives the same value, because the P1 function is continuous.  The search is brute force
over all elements, in chunks of points: plain and slow, meant for small meshes.  Points outside
the old mesh get NaN.
"""
from __future__ import annotations

import numpy as np


def evaluate_p1(X: np.ndarray, E: np.ndarray, u: np.ndarray, P: np.ndarray, tol: float = 1e-12,
                chunk: int = 512) -> np.ndarray:
    """u (values at the nodes X of the mesh with elements E) evaluated at the points P."""
    V = X[E]                                            # (ne, d+1, d)
    J = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))   # columns: edges from vertex 0
    Jinv = np.linalg.inv(J)                             # rows give lambda_1..lambda_d
    out = np.full(P.shape[0], np.nan)
    for s in range(0, P.shape[0], chunk):
        p = P[s:s + chunk]
        rel = p[:, None, :] - V[None, :, 0, :]          # (np, ne, d)
        lam = np.einsum("eij,pej->pei", Jinv, rel)     # (np, ne, d)
        full = np.concatenate([1.0 - lam.sum(axis=2, keepdims=True), lam], axis=2)
        inside = (full >= -tol).all(axis=2)             # (np, ne)
        found = inside.any(axis=1)
        e = np.argmax(inside, axis=1)
        rows = np.arange(p.shape[0])
        vals = (full[rows, e] * u[E[e]]).sum(axis=1)
        out[s:s + chunk] = np.where(found, vals, np.nan)
    return out


def transfer(h_old, u_old: np.ndarray, X_new: np.ndarray, level=None) -> np.ndarray:
    """u_old (nodal values on level L of the old hierarchy) at the new nodes X_new."""
    lv = h_old.levels[h_old.L if level is None else level]
    return evaluate_p1(lv.X, lv.E, u_old, X_new)
