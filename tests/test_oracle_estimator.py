"""Pins for the oracle's error estimator (Section 4; ErrorEstimate in Algorithm 4)."""
import os

import numpy as np
import pytest

from oracle import estimate, fmg, refine
from workloads import meshes, problems

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "effectivity_constants.txt")


def test_effectivity_constants_match_tables():
    rows = np.loadtxt(GOLDEN)
    for qn, qd, j, c1, c2 in rows:
        theta = 2.0 ** (-qn / qd)
        C1, C2 = estimate.effectivity_bounds(theta, 0.0, int(j))
        assert round(C1, 2) == pytest.approx(c1, abs=1e-9)
        assert round(C2, 2) == pytest.approx(c2, abs=1e-9)


def test_effectivity_constants_tend_to_one_and_widen_with_eps():
    C1, C2 = estimate.effectivity_bounds(0.25, 0.0, 12)
    assert abs(C1 - 1) < 1e-6 and abs(C2 - 1) < 1e-6
    a1, a2 = estimate.effectivity_bounds(0.25, 0.0, 2)
    b1, b2 = estimate.effectivity_bounds(0.25, 0.2, 2)
    assert b1 < a1 and b2 > a2


def _solve(mk, L, f_fn, g_fn, nu, smoother):
    m = mk()
    h = refine.Hierarchy(m.coords, m.cells, L)
    X = h.levels[L].X
    S = fmg.FMGSolver(h, smoother=smoother)
    b = S.rhs_levels(f_fn(X))
    g = g_fn(X)
    u, w = S.fmg(b, g, nu=nu)
    S.extra_cycles(u, b[L], g, rtol=1e-13, max_iter=100)
    return h, S, u, w, b, g


def test_local_norms_sum_to_global_and_match_quadrature():
    h, S, u, w, b, g = _solve(meshes.lshape_6tri, 4, problems.zero, problems.lshape_u, 2, "multicolour")
    est = estimate.error_estimate(S, u, w, 1)
    e = est["e_l"]
    M = S.sys[4].M
    assert abs(np.sum(est["eta_T"] ** 2) - e @ (M @ e)) < 1e-15 + 1e-12 * (e @ (M @ e))
    q = estimate.quadrature_l2(h, e, None, m=3)
    assert abs(q - est["norm_e_l"]) < 1e-12 * max(1.0, q)


def test_affine_solution_gives_zero_estimate():
    c = np.array([0.3, -1.25, 0.5])
    aff = lambda X: c[0] + X @ c[1:]
    h, S, u, w, b, g = _solve(meshes.lshape_6tri, 4, problems.zero, aff, 1, "multicolour")
    est = estimate.error_estimate(S, u, w, 1)
    assert est["norm_e_l"] < 1e-10 and est["eta_T"].max() < 1e-10


@pytest.mark.parametrize("L,nu", [(5, 2), (6, 2), (6, 6)])
def test_effectivity_within_theorem_bounds(L, nu):
    # smooth problem, q = 2, theta = 1/4, eps small once resolved: eta_1/||e_L|| in [C1, C2]
    h, S, u, w, b, g = _solve(meshes.unit_square_2tri, L, problems.sine2d_f, problems.zero, nu, "redblack")
    X = h.levels[L].X
    err = estimate.quadrature_l2(h, u, problems.sine2d_u, m=4)
    est = estimate.error_estimate(S, u, w, 1)
    C1, C2 = estimate.effectivity_bounds(0.25, 0.0, 1)
    assert C1 <= est["eta_j"] / err <= C2
    # eq. (e_tilde bounds on level L): (theta_eps^-1 - 1) <= ||e~_{L-1}|| / ||e_L|| <= theta^-1 + 1
    r = est["norm_e_l"] / err
    assert 2.5 <= r <= 5.0
    # estimated convergence factor close to 2^-2
    assert abs(est["theta"] - 0.25) < 0.06


def test_general_j_uses_prolongated_coarse_solutions():
    h, S, u, w, b, g = _solve(meshes.unit_square_2tri, 6, problems.sine2d_f, problems.zero, 2, "redblack")
    e1 = estimate.error_estimate(S, u, w, 1)
    e2 = estimate.error_estimate(S, u, w, 2)
    # j=2's e~_{l} is j=1's e~_{l-1}
    assert abs(e2["norm_e_l"] - e1["norm_e_lm1"]) < 1e-14
    assert np.allclose(e2["eta_T"], e1["eta_T"])


def test_energy_norm_matches_gradient_quadrature():
    # per macro, e^T A_T e with the macro coefficients equals int_T kappa |grad e_h|^2 computed
    # from element gradients solved directly from the nodal values; the sum is e^T A_L e
    m = meshes.lshape_6tri()
    L = 4
    h = refine.Hierarchy(m.coords, m.cells, L)
    kap = np.random.default_rng(21).uniform(0.5, 2.0, m.n_cells)
    S = fmg.FMGSolver(h, kappa_cell=kap, smoother="multicolour")
    X = h.levels[L].X
    e = np.random.default_rng(22).standard_normal(len(X))
    sq = estimate.per_macro_sq_norms(h, e, estimate.element_norm_matrices(S, "energy"))
    lv = h.levels[L]
    q = estimate.quadrature_energy(h, e, None, kappa_el=kap[lv.emacro], per_macro=True)
    assert np.allclose(sq, q, rtol=1e-12, atol=0)
    A = S.sys[L].A
    assert abs(sq.sum() - e @ (A @ e)) <= 1e-12 * sq.sum()


def test_lumped_norm_is_row_sum_diagonal_and_equivalent_to_l2():
    # lumped: sum_T ||v||_T^2 = sum_i (M 1)_i v_i^2, |Omega| for v = 1, and per macro
    # v^T M_T v <= v^T D_T v <= (d+2) v^T M_T v (eigenvalues of the P1 element mass matrix)
    for mk, L in ((meshes.lshape_6tri, 4), (lambda: meshes.kuhn_cube(1), 3)):
        m = mk()
        h = refine.Hierarchy(m.coords, m.cells, L)
        S = fmg.FMGSolver(h, smoother="redblack" if m.dim == 3 else "multicolour")
        X = h.levels[L].X
        v = np.random.default_rng(23).standard_normal(len(X))
        lum = estimate.per_macro_sq_norms(h, v, estimate.element_norm_matrices(S, "lumped"))
        con = estimate.per_macro_sq_norms(h, v, estimate.element_norm_matrices(S, "l2"))
        M = S.sys[L].M
        assert abs(lum.sum() - np.asarray(M.sum(axis=1)).ravel() @ (v * v)) <= 1e-12 * lum.sum()
        ones = estimate.per_macro_sq_norms(h, np.ones(len(X)), estimate.element_norm_matrices(S, "lumped"))
        vol = estimate.per_macro_sq_norms(h, np.ones(len(X)))
        assert np.allclose(ones, vol, rtol=1e-13)
        d = m.dim
        assert np.all(con <= lum * (1 + 1e-12)) and np.all(lum <= (d + 2) * con * (1 + 1e-12))


def test_energy_estimate_follows_galerkin_orthogonality():
    # For nested P1 spaces the energy error splits as ||e_{l}||^2 = ||e_L||^2 + ||u_L - u_l||^2
    # (Galerkin orthogonality), and P1 converges at first order in energy, ||e_l|| ~ 2^(L-l)
    # ||e_L||.  Hence ||e~_{L-1}|| / ||e_L|| -> sqrt(4 - 1) and theta~ -> sqrt(3 / 15) = 1/sqrt5
    # (not the q = 1 value 1/2: e~ of the coarser level spans two levels).  The effectivity
    # lies within the theorem's bounds for theta = 1/2.
    h, S, u, w, b, g = _solve(meshes.unit_square_2tri, 6, problems.sine2d_f, problems.zero, 2, "redblack")
    est = estimate.error_estimate(S, u, w, 1, norm="energy")
    err = estimate.quadrature_energy(h, u, problems.sine2d_grad, m=4)
    assert abs(est["theta"] - 5 ** -0.5) < 0.01
    assert abs(est["norm_e_l"] / err - 3 ** 0.5) < 0.02
    C1, C2 = estimate.effectivity_bounds(0.5, 0.0, 1)
    assert C1 <= est["eta_j"] / err <= C2
    # the L2 and lumped estimates of the same solve see second-order convergence
    assert abs(estimate.error_estimate(S, u, w, 1, norm="l2")["theta"] - 0.25) < 0.06
    assert abs(estimate.error_estimate(S, u, w, 1, norm="lumped")["theta"] - 0.25) < 0.06


@pytest.mark.parametrize("norm", ["l2", "energy", "lumped"])
def test_local_indicators_consistent_across_j(norm):
    # eta'_{j+1,T} = ||e~_{L-j-1}||_T is the denominator of theta~_{L-j,T}, so the scaled
    # indicator of j is (eta'_j / eta'_{j+1})^j eta'_j from two separate calls; the unscaled
    # indicators square-sum to ||e~_{L-j}||^2, and eta_T does not depend on j
    h, S, u, w, b, g = _solve(meshes.lshape_6tri, 5, problems.zero, problems.lshape_u, 1, "multicolour")
    for j in (1, 2, 3):
        a = estimate.error_estimate(S, u, w, j, norm=norm)
        c = estimate.error_estimate(S, u, w, j + 1, norm=norm)
        assert np.allclose(a["eta_jT"], (a["eta_prime_jT"] / c["eta_prime_jT"]) ** j * a["eta_prime_jT"],
                           rtol=1e-12, atol=0)
        assert abs(np.sum(a["eta_prime_jT"] ** 2) - a["norm_e_l"] ** 2) <= 1e-12 * a["norm_e_l"] ** 2
        assert abs(c["norm_e_l"] - a["norm_e_lm1"]) <= 1e-13 * a["norm_e_lm1"]
        assert np.allclose(a["eta_T"], estimate.error_estimate(S, u, w, 1, norm=norm)["eta_T"], rtol=1e-13)
