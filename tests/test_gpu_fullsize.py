"""GPU checks at the workloads' full sizes, where the oracle cannot run: properties that hold
at any size, plus oracle parity on the L-shape workload mesh at a level the oracle can run."""
import sys

import numpy as np
import pytest

from gpu_common import oracle_hierarchy, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def _note(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def lshape():
    from paper_2508_06049_amd import configs
    return configs.config(2)


def test_fused_sweep_equals_class_by_class_full_size(lshape):
    # the out-of-place tiled sweep must not depend on block scheduling: compare with one
    # launch per colour class on the full workload (18.9 M DoFs, thousands of tiles)
    import torch
    from paper_2508_06049_amd import HHG
    from paper_2508_06049_amd._lib import HHG_FLAG_NO_FUSED
    w = lshape
    _note("fused vs class-by-class", w.name, w.L)
    a = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother)
    X = a.dof_coords().cpu().numpy()
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal(len(X))
    b = rng.standard_normal(len(X))
    ua = to_dev(u0)
    a.smooth(w.L, ua, to_dev(b), 3)
    ra = to_host(ua)
    a.close()
    del a
    torch.cuda.synchronize()
    bb = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother, flags=HHG_FLAG_NO_FUSED)
    ub = to_dev(u0)
    bb.smooth(w.L, ub, to_dev(b), 3)
    assert rel_err(ra, to_host(ub)) < 1e-12


@pytest.mark.parametrize("L", [5, 9])
def test_lane_parallel_interface_equals_per_dof(lshape, L):
    # the lane-parallel interface sweep (one lane per DoF copy, segment sums by shuffles)
    # against the one-thread-per-DoF kernels on the workload mesh: L = 5 sweeps all classes in
    # one workgroup, L = 9 launches one grid per class
    import torch
    from paper_2508_06049_amd import HHG
    from paper_2508_06049_amd._lib import HHG_FLAG_NO_LANE_IFACE
    w = lshape
    _note("lane-parallel vs per-DoF interface", w.name, L)
    a = HHG(w.mesh.coords, w.mesh.cells, L, smoother=w.smoother)
    X = a.dof_coords().cpu().numpy()
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(len(X))
    b = rng.standard_normal(len(X))
    ua = to_dev(u0)
    a.smooth(L, ua, to_dev(b), 3)
    ra = to_host(ua)
    a.close()
    del a
    torch.cuda.synchronize()
    bb = HHG(w.mesh.coords, w.mesh.cells, L, smoother=w.smoother, flags=HHG_FLAG_NO_LANE_IFACE)
    ub = to_dev(u0)
    bb.smooth(L, ub, to_dev(b), 3)
    assert rel_err(ra, to_host(ub)) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_preloaded_interface_sweep_identical(lshape, precision):
    # the single-workgroup interface sweep that loads the sweep-invariant part of its rows
    # first sums every row in the same order as the plain form: identical solves on the
    # workload at L = 9 (small classes at every level, all classes at the coarse levels)
    import torch
    from paper_2508_06049_amd import HHG
    from paper_2508_06049_amd._lib import HHG_FLAG_NO_PRELOAD
    w = lshape
    _note("preloaded interface sweep", w.name, precision)
    out = []
    for flags in (0, HHG_FLAG_NO_PRELOAD):
        hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother, flags=flags)
        X = hh.dof_coords().cpu().numpy()
        u, st = hh.fmg_solve(to_dev(w.f(X)), to_dev(w.g(X)), nu=1, precision=precision, rtol=1e-6, max_iter=20)
        out.append((to_host(u), st.vcycles))
        hh.close()
        del hh
        torch.cuda.synchronize()
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


def test_lshape_workload_mesh_parity_at_L7(lshape):
    from oracle import fmg
    from paper_2508_06049_amd import HHG
    w = lshape
    L = 7
    _note("lshape workload mesh L7")
    h, perms = oracle_hierarchy(w.mesh, L)
    X = h.levels[L].X
    p = perms[L]
    S = fmg.FMGSolver(h, smoother=w.smoother)
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(len(X))
    b = rng.standard_normal(len(X))
    uo = u0.copy()
    S.smooth(L, uo, b, 2)
    hh = HHG(w.mesh.coords, w.mesh.cells, L, smoother=w.smoother)
    ug = to_dev(u0[p])
    hh.smooth(L, ug, to_dev(b[p]), 2)
    assert rel_err(to_host(ug), uo[p]) < 1e-12
    f, g = w.f(X), w.g(X)
    bl = S.rhs_levels(f)
    uf, _ = S.fmg(bl, g, nu=1)
    ugf, _ = hh.fmg_solve(to_dev(f[p]), to_dev(g[p]), nu=1)
    # Two float64 solvers that round differently agree only up to about cond(A_L) * eps; on
    # this graded mesh cond(A_7) ~ 2^14, i.e. ~2e-12 in the max norm.  The mass-matrix (L2)
    # norm of the difference is held to 1e-12 relative, the max norm to 4e-12.
    d = np.empty_like(uf)
    d[p] = to_host(ugf)
    d -= uf
    M = S.sys[L].M
    assert (d @ (M @ d)) ** 0.5 <= 1e-12 * (uf @ (M @ uf)) ** 0.5
    assert np.abs(d).max() <= 4e-12 * np.abs(uf).max()


def _independent_norm_e(w, hh, u_L, nu, kappa_cell=None):
    """||e~_{L-1}|| = ||u_L - P u_{L-1}||_M computed without the estimator kernels: u_{L-1} is
    the FMG solution of a context set up at level L-1 (the FMG pass up to level L-1 does not
    depend on the finer levels), P is hhg_prolongate and the norm is hhg_mass_apply."""
    import torch
    from paper_2508_06049_amd import HHG
    L = hh.L
    lo = HHG(w.mesh.coords, w.mesh.cells, L - 1, smoother=w.smoother, kappa_cell=kappa_cell)
    Xl = lo.dof_coords().cpu().numpy()
    ul, _ = lo.fmg_solve(to_dev(w.f(Xl)), to_dev(w.g(Xl)), nu=nu)
    ul = ul.clone()
    lo.close()
    del lo
    torch.cuda.synchronize()
    e = u_L - hh.prolongate(L, ul)
    return float(torch.dot(e, hh.mass_apply(e))) ** 0.5


def test_full_size_solve_converges_and_estimates(lshape):
    # properties at 18.9 M DoFs: float64 and float32-refined reach the same solution, the L2
    # error against the exact solution is stable; the estimate of the row kernel equals, per
    # macro, that of the one-thread-per-node kernel, and ||e~_{L-1}|| equals the mass norm of
    # u_L - P u_{L-1} formed from a separate level-(L-1) solve (no estimator kernel)
    import torch
    from paper_2508_06049_amd import HHG
    from paper_2508_06049_amd._lib import HHG_FLAG_GENERIC_EST
    w = lshape
    _note("full size", w.name)
    hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother)
    X = hh.dof_coords().cpu().numpy()
    f, g = to_dev(w.f(X)), to_dev(w.g(X))
    ue = to_dev(w.u_exact(X))
    u64, s64 = hh.fmg_solve(f, g, nu=1, rtol=1e-11, max_iter=60)
    est = hh.estimate(1)
    est2 = hh.estimate(2)
    u64 = u64.clone()
    un = float(torch.dot(u64, hh.mass_apply(u64))) ** 0.5
    ne = _independent_norm_e(w, hh, u64, 1)
    assert abs(ne - est["norm_e"]) <= 1e-12 * un
    hg = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother, flags=HHG_FLAG_GENERIC_EST)
    ug, _ = hg.fmg_solve(f, g, nu=1, rtol=1e-11, max_iter=60)
    assert np.array_equal(to_host(ug), to_host(u64))
    for j, ref in ((1, est), (2, est2)):
        eg = hg.estimate(j)
        assert np.abs(eg["eta_T"] - ref["eta_T"]).max() <= 1e-12 * un
        assert abs(eg["norm_e"] - ref["norm_e"]) <= 1e-12 * un
        assert abs(eg["eta_j"] - ref["eta_j"]) <= 1e-12 * un
    hg.close()
    del hg
    torch.cuda.synchronize()
    u32, s32 = hh.fmg_solve(f, g, nu=1, precision="fp32_refined", rtol=1e-11, max_iter=60)
    assert s64.final_rel_residual <= 1e-11 and s32.final_rel_residual <= 1e-11
    assert rel_err(to_host(u32), to_host(u64)) < 1e-8
    e64 = ue - u64
    err = float((e64 * hh.mass_apply(e64)).sum()) ** 0.5
    e32 = ue - u32
    err32 = float((e32 * hh.mass_apply(e32)).sum()) ** 0.5
    assert abs(err32 - err) <= 0.01 * err
    # the estimate is of the size of the error (effectivity in the range the paper reports)
    assert 0.2 < est["eta_j"] / err < 5.0


def test_lshape_estimator_drives_one_more_k_step():
    # one kl step on the L-shape workload: solve at L = 9, mark the 10 % of macros with the
    # largest eta_T, red-green refine, set up again and solve; the L2 error against the exact
    # solution drops
    import torch
    from paper_2508_06049_amd import HHG, mesh as hostmesh
    from workloads.meshes import lshape_6tri
    from workloads import problems
    rg = hostmesh.RedGreen2D(lshape_6tri())
    for _ in range(6):
        cells, _ = rg.conforming()
        origin = [v for v, q in enumerate(rg.X) if q == (0.0, 0.0)][0]
        rg.refine([i for i, c in enumerate(cells) if origin in c])
    L = 9
    errs, sizes = [], []
    marked = None
    for step in range(2):
        m = rg.mesh(f"kstep{step}")
        _note("k-step", step, m.n_cells)
        hh = HHG(m.coords, m.cells, L, smoother="multicolour")
        X = hh.dof_coords().cpu().numpy()
        g = to_dev(problems.lshape_u(X))
        f = to_dev(np.zeros(len(X)))
        u, st = hh.fmg_solve(f, g, nu=1, rtol=1e-10, max_iter=60)
        e = to_dev(problems.lshape_u(X)) - u
        errs.append(float(torch.dot(e, hh.mass_apply(e))) ** 0.5)
        sizes.append(m.n_cells)
        if step == 0:
            est = hh.estimate(1)
            eta = est["eta_T"]
            assert np.all(np.isfinite(eta)) and np.all(eta >= 0)
            marked = hostmesh.mark_fraction(eta, 0.10)
            assert len(marked) == int(np.ceil(0.1 * m.n_cells))
            assert np.min(eta[marked]) >= np.max(np.delete(eta, marked))
            rg.conforming()
            rg.refine(marked)
        hh.close()
        del hh
        torch.cuda.synchronize()
    assert sizes[1] > sizes[0]
    assert errs[1] < errs[0]


def test_cube_corner_workload_solves_and_estimates():
    # workload 4 at full size (4334 macros, L = 5): the float64 and float32-refined solves
    # agree, the error against |x|^(1/4) is small, and ||e~_{L-1}|| equals the mass norm of
    # u_L - P u_{L-1} formed without the estimator kernel
    import torch
    from paper_2508_06049_amd import HHG, configs
    w = configs.config(4)
    _note("workload 4", w.mesh.n_cells, w.L)
    hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother)
    X = hh.dof_coords().cpu().numpy()
    f, g = to_dev(w.f(X)), to_dev(w.g(X))
    u64, s64 = hh.fmg_solve(f, g, nu=1, rtol=1e-11, max_iter=60)
    est = hh.estimate(1)
    u64 = u64.clone()
    un = float(torch.dot(u64, hh.mass_apply(u64))) ** 0.5
    assert abs(_independent_norm_e(w, hh, u64, 1) - est["norm_e"]) <= 1e-12 * un
    u32, s32 = hh.fmg_solve(f, g, nu=1, precision="fp32_refined", rtol=1e-11, max_iter=60)
    assert s64.final_rel_residual <= 1e-11 and s32.final_rel_residual <= 1e-11
    assert rel_err(to_host(u32), to_host(u64)) < 1e-6
    e = to_dev(w.u_exact(X)) - u64
    err = float(torch.dot(e, hh.mass_apply(e))) ** 0.5
    assert err < 1e-3
    assert 0.0 < est["theta"] < 1.0


def test_adjoint_workload_gradient_full_size():
    # workload 5 at full size (384 macros, L = 6, 257^3 DoFs): autograd through the adjoint
    # FMG against central finite differences in two macro coefficients and along one
    # right-hand-side direction
    import torch
    from paper_2508_06049_amd import HHG, configs, hhg_solve
    from workloads import problems
    w = configs.config(5)
    _note("workload 5 adjoint", w.mesh.n_cells, w.L)
    hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother, kappa_cell=w.kappa_cell)
    X = hh.dof_coords().cpu().numpy()
    f0 = to_dev(w.f(X))
    g = to_dev(np.zeros(len(X)))
    wM = hh.mass_apply(to_dev(w.goal_weight(X)))
    opts = dict(nu=1, rtol=1e-12, max_iter=60)
    ft = f0.clone().requires_grad_(True)
    kt = torch.tensor(w.kappa_cell, dtype=torch.float64, requires_grad=True)
    torch.dot(wM, hhg_solve(hh, ft, g, kappa=kt, **opts)).backward()
    k0 = torch.tensor(w.kappa_cell, dtype=torch.float64)

    def J(fv, kv):
        with torch.no_grad():
            return float(torch.dot(wM, hhg_solve(hh, fv, g, kappa=kv, **opts)))

    gk = kt.grad.numpy()
    for e in (int(np.argmax(np.abs(gk))), 100):
        he = 1e-4 * w.kappa_cell[e]
        kp, km = k0.clone(), k0.clone()
        kp[e] += he
        km[e] -= he
        fd = (J(f0, kp) - J(f0, km)) / (2 * he)
        assert abs(fd - gk[e]) <= 1e-5 * np.abs(gk).max()
    d = to_dev(np.random.default_rng(4).standard_normal(len(X)))
    fd = (J(f0 + 1e-2 * d, k0) - J(f0 - 1e-2 * d, k0)) / 2e-2
    an = float(torch.dot(ft.grad, d))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_largest_2d_level():
    # L = 10, the largest 2D level the library sets up (n = 1024; closure coordinates take 11
    # bits), on the L-shape workload mesh: 75.5 M DoFs.  The float32-refined solve converges,
    # agrees with float64, and its error against r^(2/3) sin(2 phi/3) falls from L = 9 at
    # least as fast as the O(h) of the corner singularity
    import torch
    from paper_2508_06049_amd import HHG, configs
    w = configs.config(2)
    errs = []
    for L in (9, 10):
        _note("largest 2D level", L)
        hh = HHG(w.mesh.coords, w.mesh.cells, L, smoother=w.smoother)
        X = hh.dof_coords().cpu().numpy()
        f, g, ue = to_dev(w.f(X)), to_dev(w.g(X)), to_dev(w.u_exact(X))
        u32, s32 = hh.fmg_solve(f, g, nu=1, precision="fp32_refined", rtol=1e-10, max_iter=60)
        assert s32.final_rel_residual <= 1e-10
        if L == 10:
            assert hh.num_dofs() == 75_510_785
            u64, s64 = hh.fmg_solve(f, g, nu=1, rtol=1e-10, max_iter=60)
            assert rel_err(to_host(u32), to_host(u64)) < 1e-7
        e = ue - u32
        errs.append(float(torch.dot(e, hh.mass_apply(e))) ** 0.5)
        hh.close()
        del hh
        torch.cuda.synchronize()
    assert errs[1] < 0.55 * errs[0]


def test_largest_3d_level():
    # L = 9 on the unit cube of 6 Kuhn tetrahedra: 513^3 = 135 M DoFs, the class-by-class 3D
    # sweep at n = 512.  The solve converges in both precisions to the same solution
    import torch
    from paper_2508_06049_amd import HHG, configs
    w = configs.config(6, 9)
    _note("largest 3D level", w.mesh.n_cells, w.L)
    hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother)
    assert hh.num_dofs() == 513 ** 3
    X = hh.dof_coords().cpu().numpy()
    f, g = to_dev(w.f(X)), to_dev(w.g(X))
    u32, s32 = hh.fmg_solve(f, g, nu=1, precision="fp32_refined", rtol=1e-8, max_iter=60)
    assert s32.final_rel_residual <= 1e-8
    est = hh.estimate(1)
    assert np.all(np.isfinite(est["eta_T"])) and est["norm_e"] > 0
    u64, s64 = hh.fmg_solve(f, g, nu=1, rtol=1e-8, max_iter=60)
    assert rel_err(to_host(u32), to_host(u64)) < 1e-6


@pytest.mark.parametrize("L,precision", [(4, "fp64"), (6, "fp32_refined"), (9, "fp64"), (9, "fp32_refined")])
def test_one_launch_interface_equals_classwise(lshape, L, precision):
    # all interface classes of a 2D sweep in one launch (edge-chunk workgroups sweep the edge
    # classes, wheel workgroups the vertex classes, recomputing their edge-class neighbours)
    # against the edge and vertex classes in two launches and against one launch per class (or
    # per run of small classes): three sweeps from a random iterate, then a solve, bitwise
    # identical
    import torch
    from paper_2508_06049_amd import HHG
    from paper_2508_06049_amd._lib import HHG_FLAG_CLASSWISE_IFACE, HHG_FLAG_TWO_LAUNCH_IFACE
    w = lshape
    _note("one-launch vs classwise interface", w.name, L, precision)
    out = []
    for flags in (0, HHG_FLAG_CLASSWISE_IFACE, HHG_FLAG_TWO_LAUNCH_IFACE):
        hh = HHG(w.mesh.coords, w.mesh.cells, L, smoother=w.smoother, flags=flags)
        X = hh.dof_coords().cpu().numpy()
        rng = np.random.default_rng(7)
        ua = to_dev(rng.standard_normal(len(X)))
        hh.smooth(L, ua, to_dev(rng.standard_normal(len(X))), 3)
        u, st = hh.fmg_solve(to_dev(w.f(X)), to_dev(w.g(X)), nu=1, precision=precision, rtol=0.0, max_iter=2)
        out.append((to_host(ua), to_host(u)))
        hh.close()
        del hh
        torch.cuda.synchronize()
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0])
        assert np.array_equal(out[0][1], o[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_dense_map_and_fused_prolongation_full_size(lshape, precision):
    # the bench's step at full size (L = 9, FMG + 5 extra cycles): the dense map of levels
    # 3 .. 0 against the launches it replaces (rounding only: 1e-12 of |u| in float64; in the
    # float32-refined form the bound of the iterate test for two float32 cycles that differ in
    # rounding order, 1e-4 of the last correction), and the prolongation and zero start inside
    # the first sweeps against their own launches (bitwise)
    import torch
    from paper_2508_06049_amd import HHG
    from paper_2508_06049_amd._lib import HHG_FLAG_NO_DENSE_COARSE, HHG_FLAG_NO_FUSED_PROLONG
    w = lshape
    _note("dense map and fused prolongation at full size", w.name, w.L, precision)
    res = {}
    for name, flags, iters in (("default", 0, (5,)), ("no_dense", HHG_FLAG_NO_DENSE_COARSE, (4, 5)),
                               ("no_fused", HHG_FLAG_NO_FUSED_PROLONG, (5,))):
        hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother, flags=flags)
        X = hh.dof_coords().cpu().numpy()
        fd, gd = to_dev(w.f(X)), to_dev(w.g(X))
        for it in iters:
            u, st = hh.fmg_solve(fd, gd, nu=1, precision=precision, rtol=0.0, max_iter=it)
            res[(name, it)] = (to_host(u), st.dense_level)
        hh.close()
        del hh
        torch.cuda.synchronize()
    assert res[("default", 5)][1] == 3 and res[("no_dense", 5)][1] == -1
    assert np.array_equal(res[("default", 5)][0], res[("no_fused", 5)][0])
    a, b = res[("default", 5)][0], res[("no_dense", 5)][0]
    scale = np.abs(b).max()
    if precision == "fp64":
        tol = 1e-12 * scale
    else:
        tol = 1e-4 * np.abs(b - res[("no_dense", 4)][0]).max() + 1e-12 * scale
    assert np.abs(a - b).max() <= tol, (np.abs(a - b).max(), tol)
