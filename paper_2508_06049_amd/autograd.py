"""Differentiable HHG solve: ``u = HHGSolve.apply(f, kappa, hh, g, opts)``.

Forward: the FMG solve (plus extra cycles per ``opts``) of the per-level linear system with
right-hand side b = M f on inner rows and u = g on Dirichlet rows, for the per-macro
coefficients ``kappa`` (Section "Implementation in HyTeG", eq. of the linear system).

Backward: given the gradient of a scalar goal J with respect to the nodal solution u, the
library's adjoint solve (``hhg_adjoint``) recomputes u, solves A lambda = dJ/du with lambda = 0
on Dirichlet rows, and returns dJ/df = M lambda and dJ/dkappa_e = -lambda^T A_e u (A_e: macro
e's unit-coefficient stiffness).  Level solutions are recomputed, not kept from the forward
pass.  The gradient is that of the exact discrete solution; the solve tolerance in ``opts``
bounds how closely the computed one matches it.

The Dirichlet data g is not differentiated.  Vectors are float64 device tensors in the
library's canonical DoF order; ``kappa`` is a float64 tensor with one entry per macro (or
None to keep the context's coefficients, then no kappa gradient is returned).
"""
from __future__ import annotations

import numpy as np
import torch


class HHGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, kappa, hh, g, opts=None):
        opts = dict(opts or {})
        if kappa is not None:
            hh.set_kappa_cell(kappa.detach().to("cpu", torch.float64).numpy())
        u, _ = hh.fmg_solve(f.detach().contiguous(), g, **opts)
        ctx.hh, ctx.g, ctx.opts = hh, g, opts
        ctx.has_kappa = kappa is not None
        if kappa is not None:
            ctx.save_for_backward(f.detach(), kappa.detach())
        else:
            ctx.save_for_backward(f.detach())
        return u

    @staticmethod
    def backward(ctx, grad_u):
        saved = ctx.saved_tensors
        f = saved[0]
        kappa = saved[1] if ctx.has_kappa else None
        hh = ctx.hh
        if kappa is not None:
            # the context may have been used with other coefficients since the forward pass
            hh.set_kappa_cell(kappa.to("cpu", torch.float64).numpy())
        dJdf, dJdk = hh.adjoint(f.contiguous(), ctx.g, grad_u.detach().contiguous(), **ctx.opts)
        gf = dJdf if ctx.needs_input_grad[0] else None
        gk = None
        if kappa is not None and ctx.needs_input_grad[1]:
            gk = torch.as_tensor(np.asarray(dJdk), dtype=kappa.dtype, device=kappa.device)
        return gf, gk, None, None, None


def hhg_solve(hh, f, g, kappa=None, **opts):
    """Functional form of :class:`HHGSolve` (keyword options as for ``HHG.fmg_solve``)."""
    return HHGSolve.apply(f, kappa, hh, g, opts)
