"""Pins for the oracle's FMG (Algorithm 4, procedure FMG) against a direct sparse solve,
manufactured solutions and multigrid properties."""
import numpy as np
import pytest

from oracle import estimate, fmg, refine
from workloads import meshes, problems


def _setup(mk, L, **kw):
    m = mk()
    return refine.Hierarchy(m.coords, m.cells, L)


@pytest.mark.parametrize("mk,L,smoother,kind", [
    (meshes.unit_square_2tri, 5, "redblack", "sine"),
    (meshes.lshape_6tri, 4, "multicolour", "lshape"),
    (meshes.lshape_6tri, 4, "jacobi", "lshape"),
    (lambda: meshes.kuhn_cube(1), 4, "redblack", "fourier_kappa"),
    (lambda: meshes.kuhn_cube(2), 3, "multicolour", "fourier_kappa_cell"),
])
def test_fmg_plus_cycles_equals_direct_solve(mk, L, smoother, kind):
    h = _setup(mk, L)
    X = h.levels[L].X
    kc = kn = None
    if kind == "sine":
        f, g = problems.sine2d_f(X), np.zeros(len(X))
    elif kind == "lshape":
        f, g = np.zeros(len(X)), problems.lshape_u(X)
    elif kind == "fourier_kappa":
        f, g = problems.fourier3d(X, problems.fourier_amplitudes(0)), np.zeros(len(X))
        kn = problems.kappa_smooth3d(X)
    else:
        f, g = problems.fourier3d(X, problems.fourier_amplitudes(5)), np.zeros(len(X))
        kc = problems.kappa_cells_uniform(55, h.coarse_cells.shape[0])
    S = fmg.FMGSolver(h, kappa_cell=kc, kappa_nodal=kn, smoother=smoother)
    b = S.rhs_levels(f)
    u, w = S.fmg(b, g, nu=1)
    ud = S.direct(L, b[L], g)
    # one FMG cycle already lands within discretisation accuracy; extra cycles reach round-off
    it, rel = S.extra_cycles(u, b[L], g, rtol=1e-14, max_iter=200)
    assert np.abs(u - ud).max() <= 1e-12 * max(1.0, np.abs(ud).max())
    # w_{l} holds the prolongated level-l solution: nodes shared with level l agree with it
    for l in range(L):
        assert w[l].shape[0] == h.levels[l + 1].n


def test_vcycle_contraction():
    h = _setup(meshes.unit_square_2tri, 6)
    S = fmg.FMGSolver(h, smoother="redblack")
    X = h.levels[6].X
    rng = np.random.default_rng(0)
    b = np.zeros(len(X))
    u = rng.standard_normal(len(X))
    u[h.levels[6].boundary] = 0.0
    r0 = np.linalg.norm(S.residual(6, u, b))
    for _ in range(3):
        S.vcycle(6, u, b)
    r1 = np.linalg.norm(S.residual(6, u, b))
    assert (r1 / r0) ** (1 / 3) < 0.15


def test_mms_quadratic_convergence_unit_square():
    # optimal P1 L2 order O(h^2) (Section 5.1: O(hbar^2) for first-order elements)
    errs = []
    for L in (3, 4, 5, 6):
        h = _setup(meshes.unit_square_2tri, L)
        X = h.levels[L].X
        S = fmg.FMGSolver(h, smoother="redblack")
        b = S.rhs_levels(problems.sine2d_f(X))
        ud = S.direct(L, b[L], np.zeros(len(X)))
        errs.append(estimate.quadrature_l2(h, ud, problems.sine2d_u, m=4))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios[1:] - 4.0) < 0.1), ratios


def test_lshape_uniform_rate_four_thirds():
    # uniform refinement of the L-shape converges like O(h^(4/3)) in L2 (Section 5.2)
    errs = []
    for L in (4, 5, 6):
        h = _setup(meshes.lshape_6tri, L)
        X = h.levels[L].X
        S = fmg.FMGSolver(h, smoother="multicolour")
        g = problems.lshape_u(X)
        b = S.rhs_levels(np.zeros(len(X)))
        ud = S.direct(L, b[L], g)
        errs.append(estimate.quadrature_l2(h, ud, problems.lshape_u, m=5))
    r = errs[-2] / errs[-1]
    assert abs(np.log2(r) - 4.0 / 3.0) < 0.08, r


def test_fmg_reaches_discretisation_accuracy():
    # textbook FMG property: the FMG error is a level-independent multiple of the
    # discretisation error (one V(2,2) per level: about 1.3; two: about 1.02)
    for L in (5, 6):
        h = _setup(meshes.unit_square_2tri, L)
        X = h.levels[L].X
        S = fmg.FMGSolver(h, smoother="redblack")
        b = S.rhs_levels(problems.sine2d_f(X))
        ud = S.direct(L, b[L], np.zeros(len(X)))
        e_dir = estimate.quadrature_l2(h, ud, problems.sine2d_u)
        for nu, bound in ((1, 1.4), (2, 1.03)):
            u, _ = S.fmg(b, np.zeros(len(X)), nu=nu)
            assert estimate.quadrature_l2(h, u, problems.sine2d_u) <= bound * e_dir


def test_multigrid_is_affine_in_rhs():
    h = _setup(meshes.lshape_6tri, 3)
    S = fmg.FMGSolver(h, smoother="multicolour")
    rng = np.random.default_rng(2)
    N = h.levels[3].n
    b1, b2 = rng.standard_normal(N), rng.standard_normal(N)
    z = np.zeros(N)
    u1 = z.copy(); S.vcycle(3, u1, b1)
    u2 = z.copy(); S.vcycle(3, u2, b2)
    u3 = z.copy(); S.vcycle(3, u3, 2.0 * b1 - 3.0 * b2)
    assert np.abs(u3 - (2 * u1 - 3 * u2)).max() < 1e-12
