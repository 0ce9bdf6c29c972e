"""Helpers shared by the GPU tests: build the oracle and the HIP context for one mesh and map
between the oracle's node numbering and the library's canonical DoF order."""
from __future__ import annotations

import numpy as np

from oracle import refine


def oracle_hierarchy(mesh, L):
    h = refine.Hierarchy(mesh.coords, mesh.cells, L)
    perms = [h.canonical_order(l) for l in range(L + 1)]
    return h, perms


def hip_context(mesh, L, smoother="redblack", coefficient="macro", kappa_cell=None):
    from paper_2508_06049_amd import HHG
    return HHG(mesh.coords, mesh.cells, L, smoother=smoother, coefficient=coefficient, kappa_cell=kappa_cell)


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)
