"""GPU checks of the differentiable solve (HHGSolve): the backward pass through the library's
adjoint FMG against the oracle's adjoint gradient and against central finite differences of
the forward solve, for the goal J(u) = w^T M u with a Gaussian weight."""
import numpy as np
import pytest

from gpu_common import hip_context, oracle_hierarchy, rel_err, to_dev, to_host
from oracle import adjoint, fmg
from workloads import meshes, problems

pytestmark = pytest.mark.gpu


def _note(*a):
    print("[case]", *a, flush=True)


def _setup(m, L, seed_f=5, seed_k=55):
    h, perms = oracle_hierarchy(m, L)
    X = h.levels[L].X
    kc = problems.kappa_cells_uniform(seed_k, m.n_cells)
    f = problems.fourier3d(X, problems.fourier_amplitudes(seed_f))
    S = fmg.FMGSolver(h, kappa_cell=kc, smoother="redblack")
    Mw = S.sys[L].M @ problems.gaussian3d(X)
    return h, perms[L], X, kc, f, S, Mw


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_hhgsolve_gradient_matches_oracle(precision):
    import torch
    from paper_2508_06049_amd import hhg_solve
    m = meshes.kuhn_cube(2)
    L = 3
    _note("hhgsolve vs oracle", precision)
    h, p, X, kc, f, S, Mw = _setup(m, L)
    hh = hip_context(m, L, "redblack", kappa_cell=kc)
    opts = dict(nu=1, precision=precision, rtol=1e-14, max_iter=60)
    ft = to_dev(f[p]).requires_grad_(True)
    kt = torch.tensor(kc, dtype=torch.float64, requires_grad=True)
    g = to_dev(np.zeros(len(X)))
    u = hhg_solve(hh, ft, g, kappa=kt, **opts)
    J = torch.dot(to_dev(Mw[p]), u)
    J.backward()
    ref = adjoint.gradient(S, f, np.zeros(len(X)), Mw)
    assert rel_err(to_host(ft.grad), ref["dJdf"][p]) < 1e-10
    assert rel_err(kt.grad.numpy(), ref["dJdkappa"]) < 1e-10
    assert abs(float(J.detach()) - float(Mw @ ref["u"])) <= 1e-10 * abs(float(Mw @ ref["u"]))


def test_hhgsolve_gradient_matches_finite_differences():
    import torch
    from paper_2508_06049_amd import hhg_solve
    m = meshes.kuhn_cube(2)
    L = 3
    _note("hhgsolve vs finite differences")
    h, p, X, kc, f, S, Mw = _setup(m, L)
    hh = hip_context(m, L, "redblack", kappa_cell=kc)
    opts = dict(nu=1, rtol=1e-14, max_iter=80)
    g = to_dev(np.zeros(len(X)))
    w = to_dev(Mw[p])

    def J(fv, kv):
        with torch.no_grad():
            return float(torch.dot(w, hhg_solve(hh, fv, g, kappa=kv, **opts)))

    ft = to_dev(f[p]).requires_grad_(True)
    kt = torch.tensor(kc, dtype=torch.float64, requires_grad=True)
    torch.dot(w, hhg_solve(hh, ft, g, kappa=kt, **opts)).backward()
    f0, k0 = to_dev(f[p]), torch.tensor(kc, dtype=torch.float64)
    for e in (0, 7, 40):
        he = 1e-5 * kc[e]
        kp, km = k0.clone(), k0.clone()
        kp[e] += he
        km[e] -= he
        fd = (J(f0, kp) - J(f0, km)) / (2 * he)
        assert abs(fd - float(kt.grad[e])) <= 1e-6 * max(abs(fd), 1e-3 * float(kt.grad.abs().max()))
    d = to_dev(np.random.default_rng(2).standard_normal(len(X)))
    hf = 1e-3
    fd = (J(f0 + hf * d, k0) - J(f0 - hf * d, k0)) / (2 * hf)
    an = float(torch.dot(ft.grad, d))
    assert abs(fd - an) <= 1e-8 * abs(an)
