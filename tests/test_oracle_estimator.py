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
