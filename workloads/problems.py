"""Analytic data (right-hand sides, boundary values, coefficients, goal weights) and seeded
random parameters for the workloads.

Every function takes an (N, dim) array of points and returns (N,) float64.  These are
*inputs*: they are evaluated at node coordinates by whoever needs nodal values.  The 2D
functions of the convergence studies (sine, L-shape, waves, zero, one) also take a torch tensor
of points and then evaluate where the tensor lives, so that nodal data of a large level is made
on the device instead of on the host; so do the 3D corner problem's functions.
"""
from __future__ import annotations

import numpy as np

PI = np.pi


def _xp(x):
    """The array namespace of x: torch for tensors, numpy otherwise."""
    if type(x).__module__.startswith("torch"):
        import torch
        return torch
    return np


# --- manufactured 2D solution on the unit square: u = sin(pi x) sin(pi y) -------------------
def sine2d_u(x):
    xp = _xp(x)
    return xp.sin(PI * x[:, 0]) * xp.sin(PI * x[:, 1])


def sine2d_f(x):
    return 2.0 * PI * PI * sine2d_u(x)


def sine2d_grad(x):
    """(N, 2) gradient of sine2d_u."""
    return np.stack([PI * np.cos(PI * x[:, 0]) * np.sin(PI * x[:, 1]),
                     PI * np.sin(PI * x[:, 0]) * np.cos(PI * x[:, 1])], axis=1)


# --- L-shape corner singularity: u = r^(2/3) sin(2 phi / 3), phi in [0, 2 pi) ---------------
def lshape_u(x):
    xp = _xp(x)
    r = xp.hypot(x[:, 0], x[:, 1])
    phi = xp.arctan2(x[:, 1], x[:, 0])
    phi = xp.where(phi < 0.0, phi + 2.0 * PI, phi)
    return xp.where(r > 0.0, r ** (2.0 / 3.0) * xp.sin(2.0 * phi / 3.0), 0.0)


def zero(x):
    return _xp(x).zeros_like(x[:, 0])


def one(x):
    return _xp(x).ones_like(x[:, 0])


# --- 3D variable coefficient and seeded Fourier right-hand side ------------------------------
def kappa_smooth3d(x):
    """kappa(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z)."""
    return 1.0 + 0.5 * np.sin(2 * PI * x[:, 0]) * np.sin(2 * PI * x[:, 1]) * np.sin(2 * PI * x[:, 2])


def fourier_amplitudes(seed: int, modes: int = 8) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((modes, modes, modes))


def fourier3d(x, amplitudes: np.ndarray, chunk: int = 1 << 20):
    """f(x) = sum_{a,b,c=1..m} A_abc sin(a pi x) sin(b pi y) sin(c pi z)."""
    m = amplitudes.shape[0]
    k = np.arange(1, m + 1) * PI
    out = np.empty(x.shape[0])
    for s in range(0, x.shape[0], chunk):
        p = x[s:s + chunk]
        sx = np.sin(p[:, 0:1] * k)
        sy = np.sin(p[:, 1:2] * k)
        sz = np.sin(p[:, 2:3] * k)
        t = np.einsum("na,abc->nbc", sx, amplitudes, optimize=True)
        t = np.einsum("nbc,nb->nc", t, sy, optimize=True)
        out[s:s + chunk] = np.einsum("nc,nc->n", t, sz, optimize=True)
    return out


# --- 3D corner singularity u = |x|^alpha ------------------------------------------------------
def corner3d_u(x, alpha: float = 0.25):
    r = (x * x).sum(1) ** 0.5
    return r ** alpha


def corner3d_f(x, alpha: float = 0.25):
    """-Laplace(r^alpha) = -alpha (alpha + 1) r^(alpha - 2) in 3D; the singular node gets 0."""
    xp = _xp(x)
    r = (x * x).sum(1) ** 0.5
    v = -alpha * (alpha + 1.0) * xp.where(r > 0.0, r, 1.0) ** (alpha - 2.0)
    return xp.where(r > 0.0, v, 0.0)


# --- goal weight: Gaussian bump ---------------------------------------------------------------
def gaussian3d(x, center=(0.5, 0.5, 0.5), sigma: float = 0.1):
    d2 = np.sum((x - np.asarray(center)) ** 2, axis=1)
    return np.exp(-d2 / (2.0 * sigma * sigma))


def kappa_cells_uniform(seed: int, n: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


# --- 2D "waves" problem: u = w(x) w(y), w(t) = 1 - cos(exp(a (t-1)) om t) ---------------------
def waves_w(t, om=16 * PI, a=10.0):
    xp = _xp(t)
    return 1.0 - xp.cos(xp.exp(a * (t - 1.0)) * om * t)


def waves_w2(t, om=16 * PI, a=10.0):
    """Second derivative of w."""
    xp = _xp(t)
    e = xp.exp(a * (t - 1.0))
    th = e * om * t
    th1 = om * e * (1.0 + a * t)
    th2 = om * e * a * (2.0 + a * t)
    return xp.cos(th) * th1 * th1 + xp.sin(th) * th2


def waves_u(x, om=16 * PI, a=10.0):
    u = waves_w(x[:, 0], om, a)
    for i in range(1, x.shape[1]):
        u = u * waves_w(x[:, i], om, a)
    return u


def waves_f(x, om=16 * PI, a=10.0):
    d = x.shape[1]
    w = [waves_w(x[:, i], om, a) for i in range(d)]
    w2 = [waves_w2(x[:, i], om, a) for i in range(d)]
    f = zero(x)
    for i in range(d):
        t = w2[i]
        for k in range(d):
            if k != i:
                t = t * w[k]
        f = f - t
    return f
