"""kl-refinement loop (Section 3, Algorithm "kl-Refinement") on the GPU against the oracle: at
every step the per-macro criterion (local errors against the exact solution, or the estimator
eta_T), the global error and the level-0 error match the oracle on the same macro mesh, and
the marked set is the one the oracle's values select (where values tie within the tolerance,
any of the tied macros is a valid choice, so only the separated ones are compared)."""
import math

import numpy as np
import pytest

from oracle import estimate, fmg, refine
from workloads import meshes, problems

pytestmark = pytest.mark.gpu


def _note(*a):
    print("[case]", *a, flush=True)


def _oracle(mesh, L, f, g, u, nu, smoother):
    h = refine.Hierarchy(mesh.coords, mesh.cells, L)
    X = h.levels[L].X
    S = fmg.FMGSolver(h, smoother=smoother)
    b = S.rhs_levels(f(X))
    gg = g(X)
    uo, wo = S.fmg(b, gg, nu=nu)
    S.extra_cycles(uo, b[L], gg, rtol=1e-13, max_iter=200)
    ue = u(X)
    sq = estimate.per_macro_sq_norms(h, ue - uo)
    sq0 = estimate.per_macro_sq_norms(h, ue - estimate.prolongate_to(S, wo[0], 1, L))
    eta_T = estimate.error_estimate(S, uo, wo, 1)["eta_T"]
    eta = {j: estimate.error_estimate(S, uo, wo, j)["eta_j"] for j in range(1, L)}
    scale = math.sqrt(uo @ (S.sys[L].M @ uo))
    return sq, sq0, eta_T, eta, scale


CASES = {
    # Section 5.1: waves problem on the 32-triangle unit square, refinement by local errors
    "waves": (meshes.unit_square_grid(4), problems.waves_f, problems.zero, problems.waves_u, "error", 4, 3),
    # Section 5.2: L-shape on 24 triangles, here driven by the estimator
    "lshape24": (meshes.lshape_24tri(), problems.zero, problems.lshape_u, problems.lshape_u, "estimate", 4, 3),
    # tetrahedra: the corner singularity |x|^(1/4) on the 6-tetrahedron cube, by the estimator
    # and (warm-started) by local errors
    "corner3d": (meshes.kuhn_cube(1), problems.corner3d_f, problems.corner3d_u, problems.corner3d_u, "estimate", 3, 2),
    "corner3d_err": (meshes.kuhn_cube(1), problems.corner3d_f, problems.corner3d_u, problems.corner3d_u, "error", 3, 2),
}


@pytest.mark.parametrize("name,warm", [("waves", False), ("lshape24", False), ("waves", True), ("corner3d", False),
                                       ("corner3d_err", True)])
def test_kl_loop_matches_oracle(name, warm):
    # warm: steps after the first start from the transferred solution of the previous step
    from paper_2508_06049_amd import kl
    coarse, f, g, u, crit, L, K = CASES[name]
    nu = 2
    js = tuple(range(1, min(L, 4)))
    _note("kl loop", name, crit, L, K, "warm" if warm else "fmg")
    steps = kl.kl_refine(coarse, L, K, f, g, u, criterion=crit, nu=nu, rtol=1e-13, max_iter=200, tighten=0,
                         warm=warm, estimate_js=js)
    assert len(steps) == K + 1
    for s in steps:
        sq, sq0, eta_T, eta, scale = _oracle(s.mesh, L, f, g, u, nu, "multicolour")
        tol = 1e-12 * scale
        ref = np.sqrt(sq) if crit == "error" else eta_T
        assert np.all(np.abs(s.local - ref) <= tol)
        assert abs(s.err - math.sqrt(sq.sum())) <= tol
        if warm and s.k > 0:
            assert s.err_level0 is None and s.extra["transfer_s"] > 0 and not s.extra["eta"]
        else:
            assert abs(s.err_level0 - math.sqrt(sq0.sum())) <= tol
            assert sorted(s.extra["eta"]) == list(js)
            for j in js:
                assert abs(s.extra["eta"][j] - eta[j]) <= tol
        if s.marked is None:
            continue
        n = s.n_macros
        assert len(s.marked) == math.ceil(0.1 * n) and len(set(s.marked.tolist())) == len(s.marked)
        thr = np.sort(ref)[::-1][len(s.marked) - 1]
        assert np.all(ref[s.marked] >= thr - 2 * tol)
        assert set(np.nonzero(ref > thr + 2 * tol)[0].tolist()) <= set(s.marked.tolist())
    sizes = [s.n_macros for s in steps]
    assert all(b > a for a, b in zip(sizes, sizes[1:]))
    assert steps[-1].err < steps[0].err
    rho = kl.error_ratio(steps)
    assert all(np.isfinite(rho))
