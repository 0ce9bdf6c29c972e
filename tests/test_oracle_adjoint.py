"""Pins for the oracle's adjoint gradient: duality and finite differences."""
import numpy as np

from oracle import adjoint, assemble, fmg, refine
from workloads import meshes, problems


def _setup(L=2, ns=2):
    m = meshes.kuhn_cube(ns)
    h = refine.Hierarchy(m.coords, m.cells, L)
    kc = problems.kappa_cells_uniform(55, h.coarse_cells.shape[0])
    X = h.levels[L].X
    f = problems.fourier3d(X, problems.fourier_amplitudes(5))
    wg = problems.gaussian3d(X)
    return h, kc, X, f, wg


def _J(h, kc, f, wg):
    S = fmg.FMGSolver(h, kappa_cell=kc, smoother="redblack")
    M = S.sys[h.L].M
    b = M @ f
    u = S.direct(h.L, b, np.zeros(len(f)))
    return float(wg @ (M @ u)), S, M


def test_duality():
    h, kc, X, f, wg = _setup()
    J, S, M = _J(h, kc, f, wg)
    out = adjoint.gradient(S, f, np.zeros(len(f)), M @ wg)
    b = M @ f
    inner = ~h.levels[h.L].boundary
    assert abs(J - float(out["lam"][inner] @ b[inner])) < 1e-12 * abs(J)
    # dJ/df is exact because J is linear in f
    assert abs(J - float(out["dJdf"] @ f)) < 1e-12 * abs(J)


def test_finite_differences_f_and_kappa():
    h, kc, X, f, wg = _setup()
    J0, S, M = _J(h, kc, f, wg)
    out = adjoint.gradient(S, f, np.zeros(len(f)), M @ wg)
    rng = np.random.default_rng(7)
    eps = 1e-6
    for i in rng.choice(len(f), 4, replace=False):
        fp, fm = f.copy(), f.copy()
        fp[i] += eps; fm[i] -= eps
        fd = (_J(h, kc, fp, wg)[0] - _J(h, kc, fm, wg)[0]) / (2 * eps)
        assert abs(fd - out["dJdf"][i]) <= 1e-6 * np.abs(out["dJdf"]).max()
    for e in rng.choice(len(kc), 4, replace=False):
        kp, km = kc.copy(), kc.copy()
        kp[e] += eps; km[e] -= eps
        fd = (_J(h, kp, f, wg)[0] - _J(h, km, f, wg)[0]) / (2 * eps)
        assert abs(fd - out["dJdkappa"][e]) <= 1e-5 * abs(out["dJdkappa"][e]) + 1e-12
