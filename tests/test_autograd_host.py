"""Host check of the differentiable solve's wiring (HHGSolve): forward and backward are driven
through a CPU stand-in with the library's method names, whose solves and adjoint are the
oracle's, and torch.autograd.gradcheck compares the backward pass with finite differences of
the forward pass in f and in the per-macro coefficients."""
import numpy as np
import pytest
import torch

from oracle import adjoint, fmg, refine
from workloads import meshes, problems


class OracleContext:
    """CPU stand-in for paper_2508_06049_amd.HHG: canonical-order vectors, exact solves."""

    def __init__(self, mesh, L):
        self.h = refine.Hierarchy(mesh.coords, mesh.cells, L)
        self.L = L
        self.perm = self.h.canonical_order(L)
        self.kc = np.ones(mesh.n_cells)
        self._S = None

    def set_kappa_cell(self, k):
        k = np.asarray(k, dtype=np.float64)
        if self._S is None or not np.array_equal(k, self.kc):
            self.kc = k.copy()
            self._S = None

    def _solver(self):
        if self._S is None:
            self._S = fmg.FMGSolver(self.h, kappa_cell=self.kc)
        return self._S

    def _to_oracle(self, v):
        o = np.empty(len(self.perm))
        o[self.perm] = v.detach().numpy()
        return o

    def fmg_solve(self, f, g, **kw):
        S = self._solver()
        s = S.sys[self.L]
        u = S.direct(self.L, s.M @ self._to_oracle(f), self._to_oracle(g))
        return torch.as_tensor(u[self.perm]), None

    def adjoint(self, f, g, dJdu, **kw):
        r = adjoint.gradient(self._solver(), self._to_oracle(f), self._to_oracle(g), self._to_oracle(dJdu))
        return torch.as_tensor(r["dJdf"][self.perm]), r["dJdkappa"]


@pytest.mark.parametrize("mk,L", [(meshes.lshape_6tri, 2), (lambda: meshes.kuhn_cube(1), 2)])
def test_hhgsolve_gradcheck(mk, L):
    from paper_2508_06049_amd.autograd import HHGSolve
    m = mk()
    ctx = OracleContext(m, L)
    X = ctx.h.levels[L].X[ctx.perm]
    rng = np.random.default_rng(3)
    f = torch.tensor(rng.standard_normal(len(X)), requires_grad=True)
    g = torch.tensor(np.where(np.isin(np.arange(len(X)), np.nonzero(ctx.h.levels[L].boundary[ctx.perm])[0]),
                              X[:, 0] + 0.5, 0.0))
    k = torch.tensor(rng.uniform(0.5, 2.0, m.n_cells), requires_grad=True)
    assert torch.autograd.gradcheck(lambda f_, k_: HHGSolve.apply(f_, k_, ctx, g, {}), (f, k), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)


def test_hhgsolve_goal_gradient_matches_oracle_adjoint():
    # J(u) = w^T M u: the autograd gradient equals the oracle's adjoint gradient
    from paper_2508_06049_amd.autograd import hhg_solve
    m = meshes.kuhn_cube(2)
    L = 2
    ctx = OracleContext(m, L)
    S0 = fmg.FMGSolver(ctx.h)
    X = ctx.h.levels[L].X
    Mw = S0.sys[L].M @ problems.gaussian3d(X)
    fo = problems.fourier3d(X, problems.fourier_amplitudes(5))
    kc = problems.kappa_cells_uniform(55, m.n_cells)
    p = ctx.perm
    f = torch.tensor(fo[p], requires_grad=True)
    k = torch.tensor(kc, requires_grad=True)
    g = torch.zeros(len(X), dtype=torch.float64)
    u = hhg_solve(ctx, f, g, kappa=k)
    J = torch.dot(torch.as_tensor(Mw[p]), u)
    J.backward()
    ref = adjoint.gradient(fmg.FMGSolver(ctx.h, kappa_cell=kc), fo, np.zeros(len(X)), Mw)
    assert np.abs(f.grad.numpy() - ref["dJdf"][p]).max() <= 1e-12 * np.abs(ref["dJdf"]).max()
    assert np.abs(k.grad.numpy() - ref["dJdkappa"]).max() <= 1e-12 * np.abs(ref["dJdkappa"]).max()
