#!/usr/bin/env python3
"""Benchmark of the HHG full-multigrid hot path on one MI355X.

Workload (default): the L-shape domain with its 6 macro triangles k-refined 6 times towards
the re-entrant corner (144 macros), L = 9 structured levels (18.9 M DoFs), Dirichlet data
u = r^(2/3) sin(2 phi / 3), f = 0, multicolour Gauss-Seidel V(2,2), one V-cycle per FMG
level.  One step = one FMG solve to the fixed discretisation-level L2 error + the error
estimate of every macro element.

The fixed error: the discrete L2 (mass-matrix) norm of I_L u - u_h is computed for a solve
converged to a relative residual of 1e-12 (float64); each precision then runs the FMG pass and
the smallest number of extra V-cycles whose error is within 1 % of that value (calibration, not
timed; the timed solves compute no residual norms).  `value` is the whole-job DoF/s of the float32-refined path; the float64 path is
reported beside it.  The smoother's bandwidth is measured separately on level L, and the
roofline entry uses the finest-level interior smoother kernel (float32), timed per launch
with HIP events on the library's stream.

cpu_baseline: the CPU oracle (assembled sparse matrices, same FMG, same colouring and
smoother) on the same mesh at L = 7, solved to its own fixed error at that level (the same
stopping rule: FMG and the fewest extra cycles within 1 % of the converged error), on one host
core and on every host core at once (one process each), before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30          # plain copy used to scale the HBM byte counters
# HBM bytes per launch of the finest-level float32 sweep on the L-shape workload (L = 9), from
# FETCH_SIZE and WRITE_SIZE counter runs of `bench.py --kernel-only`, each scaled by the same
# counter's reading for a 1 GiB device copy (fetch x2.000, write x1.000); valid for the kernel
# as committed with profiles/k_gs2d_fused_lshape_L9_traffic.md, else reported as null
TRAFFIC_BYTES = {("lshape_corner", 9, "k_gs2d_fused<float, 3, 18, 1, true, 0>"): 228.5e6}
# the finest-level interior smoother kernel per workload type (float32 sweeps)
KERNEL_NAME = {
    (2, "multicolour", "macro"): "k_gs2d_fused<float, 3, 18, 1, true, 0>",
    (2, "redblack", "macro"): "k_gs2d_fused<float, 2, 16, 1, true, 0>",
    (3, "multicolour", "macro"): "k_gs3d_macro<float, 4, true>",
    (3, "redblack", "macro"): "k_gs3d_macro<float, 2, true>",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def l2_error(hh, u, u_ex):
    e = u_ex - u
    return math.sqrt(float((e * hh.mass_apply(e)).sum()))


def calibrate(hh, f, g, u_ex, w, precision, e_ref, kmax=60):
    """The smallest number k of extra V-cycles after the FMG pass whose L2 error is within 1 % of
    the converged one (the fixed error of the metric); the timed solves then run FMG + k cycles
    with no residual norms (rtol = 0)."""
    for k in range(kmax + 1):
        u, st = hh.fmg_solve(f, g, nu=w.nu, pre=w.pre, post=w.post, precision=precision, rtol=0.0, max_iter=k)
        err = l2_error(hh, u, u_ex)
        if err <= 1.01 * e_ref:
            return k, err, st
    raise RuntimeError(f"{precision}: no extra-cycle count up to {kmax} reaches 1.01 x {e_ref:.4e}")


def timed_steps(hh, f, g, w, precision, extra, steps, warmup, rtol=0.0):
    import torch
    for _ in range(warmup):
        hh.fmg_solve(f, g, nu=w.nu, pre=w.pre, post=w.post, precision=precision, rtol=rtol, max_iter=extra)
        hh.estimate(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        _, st = hh.fmg_solve(f, g, nu=w.nu, pre=w.pre, post=w.post, precision=precision, rtol=rtol, max_iter=extra)
        est = hh.estimate(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, st, est


def _oracle_solver(w, L):
    from oracle import fmg, refine
    h = refine.Hierarchy(w.mesh.coords, w.mesh.cells, L)
    S = fmg.FMGSolver(h, smoother=w.smoother, nu1=w.pre, nu2=w.post)
    X = h.levels[L].X
    return h, S, S.rhs_levels(w.f(X)), w.g(X), X


def _oracle_timed(S, b, g, L, nu, extra, seconds):
    reps, t = 0, 0.0
    while t < seconds:
        t0 = time.perf_counter()
        u, _ = S.fmg(b, g, nu=nu)
        if extra:
            S.extra_cycles(u, b[L], g, rtol=1e-300, max_iter=extra)
        t += time.perf_counter() - t0
        reps += 1
    return reps, t


def _oracle_worker(args):
    """One host core: set up the oracle and time solves for `seconds` (spawned process)."""
    cfg, L_, extra, seconds = args
    from paper_2508_06049_amd import configs
    w = configs.config(cfg)
    h, S, b, g, _ = _oracle_solver(w, L_)
    reps, t = _oracle_timed(S, b, g, L_, w.nu, extra, seconds)
    return h.levels[L_].n * reps, t


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    # at most 16 workers: the host share of one GPU on the measurement machines
    return max(1, min(n, 16))


def cpu_baseline(w, cfg, L=7, seconds=8.0):
    """The oracle, as it stands, on the same macro mesh at L = 7: its own fixed error (the
    converged float64 discretisation error at that level, against the exact solution when one
    is known), the fewest extra cycles after FMG within 1 % of it, then such solves timed on one
    core (median of 3 runs of `seconds` each) and on every host core at once (one process per
    core, each solving the same problem).  Assembly excluded.
    Must run before this process touches the GPU (its workers are spawned processes)."""
    import multiprocessing as mp
    import numpy as np
    t_setup = time.perf_counter()
    h, S, b, g, X = _oracle_solver(w, L)
    t_setup = time.perf_counter() - t_setup
    M = S.sys[L].M
    ud = S.direct(L, b[L], g)
    uex = w.u_exact(X) if w.u_exact is not None else ud
    err = lambda u: float(np.sqrt((uex - u) @ (M @ (uex - u))))
    e_ref = err(ud)
    # the same stopping rule as on the GPU: the smallest number of extra cycles after FMG whose
    # error is within 1 % of the converged one (without an exact solution the reference is the
    # discrete solution itself, and the count whose error falls below 1e-6 of it is taken)
    u, _ = S.fmg(b, g, nu=w.nu)
    extra = 0
    while err(u) > max(1.01 * e_ref, 1e-6 * float(np.sqrt(ud @ (M @ ud)))) and extra < 60:
        S.extra_cycles(u, b[L], g, rtol=1e-300, max_iter=1)
        extra += 1
    n = h.levels[L].n
    one = []
    for _ in range(3):
        reps, t = _oracle_timed(S, b, g, L, w.nu, extra, seconds / 3)
        one.append(n * reps / t)
    v1 = float(np.median(one))
    del S, h
    cores = host_cores()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(cfg, L, extra, seconds)] * cores)
    vN = sum(d / t for d, t in res)
    return dict(value=vN, unit="DoF/s", cores=cores, kind="oracle", cpu_model=host_cpu_model(),
                single_core=dict(value=v1, cores=1, median_of=3),
                sample=f"{w.name} macro mesh at L={L} ({n} DoFs): float64 FMG nu={w.nu} V({w.pre},{w.post}) "
                       f"{w.smoother} + {extra} extra cycles, the fewest whose L2 error is within 1 % of "
                       f"the converged one at L={L} ({e_ref:.4e}); one core: median of 3; all cores: {cores} "
                       f"processes, each timing its own solves for {seconds:g} s; assembly ({t_setup:.1f} s) excluded; "
                       f"scipy sparse, one thread per process")


def step_algorithmic_bytes(ndofs, dim, nu, pre, post, fmg_cycles, extra_cycles, precision, norms=True):
    """Bytes the method must move per step (one FMG solve with its extra cycles, the right-hand
    sides and the estimate) with every kernel at its ideal traffic: a smoother sweep moves
    3 s bytes per DoF (s = 8 float64, 4 float32), a residual fused with the restriction
    2 s + s/2^d, a prolongation-add 2 s + s/2^d, the FMG prolongation with the w store
    16 + 8/2^d, the float32-refined fine residual and update 20 each, the estimate
    16 + 8/2^d, a right-hand side b_l = M_l f_l 16 per DoF of its level, the canonical-order
    conversion of f, g and u 16 per level-L DoF each.  ndofs[l]: DoFs of level l."""
    c = 1.0 / 2 ** dim

    def vcyc(l, s):
        tot = 0.0
        for k in range(l, 0, -1):
            tot += ndofs[k] * ((pre + post) * 3 * s + 2 * (2 * s + s * c))
        return tot

    def cyc(l):
        if precision == "fp64":
            return vcyc(l, 8)
        return ndofs[l] * 40 + vcyc(l, 4)

    L = len(ndofs) - 1
    b = sum(16.0 * n for n in ndofs) + 3 * 16.0 * ndofs[L]
    for l in range(1, L + 1):
        b += ndofs[l] * (16 + 8 * c) + nu * cyc(l)
    norm = (32.0 if precision == "fp64" else 4.0) if norms else 0.0
    b += extra_cycles * (cyc(L) + norm * ndofs[L])
    b += ndofs[L] * (16 + 8 * c)
    return b


# convergence studies of Section 5 (coarse mesh, f, g, u, criterion): the waves problem on the
# 32-triangle unit square (Section 5.1) and the L-shape on 24 triangles (Section 5.2), both
# refined by the actual local errors, 10 % of the macros per step
KL_CASES = {
    "waves": ("unit_square_grid4", "waves_f", "zero", "waves_u"),
    "lshape24": ("lshape_24tri", "zero", "lshape_u", "lshape_u"),
}


def run_kl(args):
    from paper_2508_06049_amd import kl
    from workloads import meshes, problems

    mname, fn, gn, un = KL_CASES[args.kl]
    coarse = meshes.unit_square_grid(4) if mname == "unit_square_grid4" else getattr(meshes, mname)()
    f, g, u = getattr(problems, fn), getattr(problems, gn), getattr(problems, un)
    K, L = args.kl_K, args.kl_L
    log(f"kl loop {args.kl}: {coarse.n_cells} macros, K={K}, L={L}")

    def show(s):
        e0 = "-" if s.err_level0 is None else f"{s.err_level0:.4e}"
        log(f"k={s.k}: {s.n_macros} macros, {s.n_dofs} DoFs, error {s.err:.4e}, level-0 error {e0}, "
            f"transfer {s.extra['transfer_s'] * 1e3:.1f} ms, {s.vcycles} V-cycles ({s.extra['solves']} solves, "
            f"rel. residual {s.extra['final_rel_residual']:.1e}), "
            f"setup {s.t_setup:.2f} s, solve {s.t_solve * 1e3:.1f} ms, local norms "
            f"{s.t_local * 1e3:.1f} ms, mark+refine {s.t_refine * 1e3:.1f} ms")

    t0 = time.perf_counter()
    steps = kl.kl_refine(coarse, L, K, f, g, u, criterion="error", nu=2, rtol=1e-6, max_iter=100, callback=show,
                         warm=args.kl_warm)
    t_loop = time.perf_counter() - t0
    rho = kl.error_ratio(steps)
    # uniform refinement of T_0^0 (levels 1..L), same solver and stopping rule
    H = kl.mean_width(coarse, 0)
    uni = []
    for l in range(1, L + 1):
        s = kl.kl_refine(coarse, l, 0, f, g, u, criterion="error", nu=2, rtol=1e-6, max_iter=100)[0]
        uni.append(dict(L=l, dofs=s.n_dofs, error=s.err, rho=H * H * s.err / (s.hbar * s.hbar * steps[0].err_level0)))
        log(f"uniform L={l}: {s.n_dofs} DoFs, error {s.err:.4e}, rho {uni[-1]['rho']:.3f}")
    out = {
        "metric": "kl-refinement loop: error ratio rho and time per k-step",
        "value": rho[-1], "unit": "rho on T_L^K", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "config": {"workload": f"kl_{args.kl}", "coarse_macros": coarse.n_cells, "K": K, "L": L,
                   "start": "transferred solution + V-cycles" if args.kl_warm else "FMG",
                   "marking": "10 % largest local L2 errors, red-green", "smoother": "multicolour", "fmg_nu": 2,
                   "vcycle": [2, 2], "rtol": "1e-6, lowered 100-fold until the error's first two digits are stable"},
        "loop_seconds": round(t_loop, 3),
        "steps": [dict(k=s.k, macros=s.n_macros, dofs=s.n_dofs, error=s.err, level0_error=s.err_level0,
                       rho=r, eta_1=s.eta_1, vcycles=s.vcycles, solves=s.extra["solves"], setup_s=round(s.t_setup, 4),
                       solve_ms=round(s.t_solve * 1e3, 3), local_ms=round(s.t_local * 1e3, 3),
                       refine_ms=round(s.t_refine * 1e3, 3), transfer_ms=round(s.extra["transfer_s"] * 1e3, 3))
                  for s, r in zip(steps, rho)],
        "uniform": uni,
    }
    print(json.dumps(out), flush=True)


def run_kl_study(args):
    """Section 5.3: effectivity gamma_j = eta_j / ||e|| (j = 1..4) over the kl sequence refined
    by local errors, with nu = 6, 2, 1 V-cycles per FMG level (worst case over k per j); then
    the kl loop refined by eta_T computed with nu = 1, 2, 6, against refinement by the errors."""
    from paper_2508_06049_amd import kl
    from workloads import meshes, problems

    mname, fn, gn, un = KL_CASES[args.kl]
    coarse = meshes.unit_square_grid(4) if mname == "unit_square_grid4" else getattr(meshes, mname)()
    f, g, u = getattr(problems, fn), getattr(problems, gn), getattr(problems, un)
    K, L = args.kl_K, args.kl_L
    js = [j for j in (1, 2, 3, 4) if j < L]
    out = {"metric": "estimator effectivity eta_j/||e|| and kl refinement by eta_T, per nu",
           "unit": "ratio", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"kl_{args.kl}", "coarse_macros": coarse.n_cells, "K": K, "L": L,
                      "smoother": "multicolour", "vcycle": [2, 2], "marking": "10 %, red-green"},
           "effectivity": {}, "indicator": {}}
    t0 = time.perf_counter()
    for nu in (6, 2, 1):
        steps = kl.kl_refine(coarse, L, K, f, g, u, criterion="error", nu=nu, rtol=1e-6, max_iter=100,
                             estimate_js=js)
        worst = {j: kl.worst_effectivity(steps, j) for j in js}
        out["effectivity"][f"nu{nu}"] = {
            "gamma": {j: kl.effectivity(steps, j) for j in js},
            "worst": {j: dict(k=k, gamma=gm) for j, (k, gm) in worst.items()}}
        log(f"nu={nu}: worst effectivity " + ", ".join(f"j={j}: {gm:.2f} (k={k})" for j, (k, gm) in worst.items()))
    ref = None
    for nu in ("error", 1, 2, 6):
        crit = "error" if nu == "error" else "estimate"
        steps = kl.kl_refine(coarse, L, K, f, g, u, criterion=crit, nu=2 if nu == "error" else nu, rtol=1e-6,
                             max_iter=100)
        rho = kl.error_ratio(steps)
        out["indicator"]["errors" if nu == "error" else f"eta_T_nu{nu}"] = dict(
            macros=[s.n_macros for s in steps], dofs=[s.n_dofs for s in steps], error=[s.err for s in steps],
            rho=rho)
        log(f"refined by {'local errors' if nu == 'error' else f'eta_T with nu={nu}'}: final error "
            f"{steps[-1].err:.3e}, rho {rho[-1]:.2f}, {steps[-1].n_macros} macros")
    out["seconds"] = round(time.perf_counter() - t0, 2)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the smoother sweeps on level L and a plain device copy of known size "
                         "(for hardware-counter runs; prints no JSON line)")
    ap.add_argument("--flags", type=int, default=0,
                    help="hhg_options.flags of the context (e.g. 1: class-by-class interior sweeps) for A/B timing")
    ap.add_argument("--kernel-only-fp64", action="store_true",
                    help="with --kernel-only: also time float64 sweeps")
    ap.add_argument("--profile-step", choices=["fp64", "fp32_refined"], default=None,
                    help="run only --warmup and --steps steps of one precision (FMG + --extra cycles, the "
                         "estimate), without calibration or baseline, for kernel traces of the step alone; "
                         "prints the ms per step, no JSON line")
    ap.add_argument("--extra", type=int, default=5, help="with --profile-step: extra cycles after FMG")
    ap.add_argument("--kl", choices=sorted(KL_CASES), default=None,
                    help="run the kl-refinement loop (Section 3) on one of the convergence-study problems of "
                         "Section 5 instead of the solve benchmark, with a uniform-refinement baseline; prints "
                         "one JSON line")
    ap.add_argument("--kl-K", type=int, default=10)
    ap.add_argument("--kl-L", type=int, default=8)
    ap.add_argument("--kl-study", action="store_true",
                    help="with --kl: the estimator study of Section 5.3 (effectivity of eta_j for nu = 6, 2, 1 "
                         "and refinement by eta_T for nu = 1, 2, 6); prints one JSON line")
    ap.add_argument("--kl-warm", action="store_true",
                    help="kl loop: start each step after the first from the transferred solution of the "
                         "previous step (hhg_transfer + hhg_cycle_solve) instead of an FMG solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the method runs on one GPU here); --gpus {args.gpus} is not "
              f"supported", file=sys.stderr)
        sys.exit(2)
    if args.kl:
        run_kl_study(args) if args.kl_study else run_kl(args)
        return

    from paper_2508_06049_amd import configs
    cpu = None
    if not args.no_cpu_baseline and not args.kernel_only and not args.profile_step:
        # the oracle runs first: its worker processes start before this process touches the GPU
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(configs.config(args.config), args.config)
        log(f"cpu baseline: {cpu['value']:.3e} DoF/s on {cpu['cores']} cores, "
            f"{cpu['single_core']['value']:.3e} DoF/s on one ({cpu['cpu_model']})")

    import numpy as np
    import torch
    from paper_2508_06049_amd import HHG

    if args.config == 3:
        print("bench.py: workload 3 needs the nodal-coefficient path, which is switched off in this build "
              "(a parity run of it ended in a GPU memory fault whose cause was not found)", file=sys.stderr)
        sys.exit(2)
    w = configs.config(args.config, args.L)
    log(f"workload {w.name}: {w.mesh.n_cells} macros, L={w.L}, smoother {w.smoother}")
    hh = HHG(w.mesh.coords, w.mesh.cells, w.L, smoother=w.smoother, coefficient=w.coefficient,
             kappa_cell=w.kappa_cell, flags=args.flags)
    N = hh.num_dofs()
    X = hh.dof_coords().cpu().numpy()
    if w.kappa_nodal is not None:
        hh.set_kappa_nodal(torch.as_tensor(w.kappa_nodal(X), device="cuda:0"))
    log(f"N = {N} DoFs, workspace {hh.workspace_bytes / 2**30:.2f} GiB")
    if args.kernel_only:
        # counter calibration: a device-to-device copy of COPY_BYTES, then the float32 sweeps
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        hh.bench_smoother("fp32_refined", 2)   # first touch of the level's pages
        b = hh.bench_smoother("fp32_refined", args.sweeps)
        log(f"kernel-only: copy of {COPY_BYTES} B x3, {args.sweeps} float32 sweeps, interior launch "
            f"{b['launch_ms'] * 1e3:.1f} us, {b['launch_bytes']:.0f} algorithmic bytes per launch "
            f"({b['launch_bytes'] / (b['launch_ms'] * 1e-3) / 1e9:.0f} GB/s)")
        if args.kernel_only_fp64:
            hh.bench_smoother("fp64", 2)
            b = hh.bench_smoother("fp64", args.sweeps)
            log(f"kernel-only: {args.sweeps} float64 sweeps, interior launch {b['launch_ms'] * 1e3:.1f} us "
                f"({b['launch_bytes'] / (b['launch_ms'] * 1e-3) / 1e9:.0f} GB/s)")
        return

    f = torch.as_tensor(w.f(X), device="cuda:0")
    g = torch.as_tensor(w.g(X), device="cuda:0")
    if args.profile_step:
        ms, st, _ = timed_steps(hh, f, g, w, args.profile_step, args.extra, args.steps, args.warmup)
        log(f"profile step {args.profile_step}: FMG + {args.extra} extra cycles, {st.vcycles} V-cycles, "
            f"{ms:.3f} ms per step over {args.steps} steps")
        return
    # reference discretisation error: converged float64 solve
    u_ref, st_ref = hh.fmg_solve(f, g, nu=w.nu, pre=w.pre, post=w.post, precision="fp64", rtol=1e-12, max_iter=200)
    if w.u_exact is not None:
        u_ex = torch.as_tensor(w.u_exact(X), device="cuda:0")
    else:
        u_ex = u_ref.clone()
    e_ref = l2_error(hh, u_ref, u_ex)
    log(f"converged float64: {st_ref.vcycles} V-cycles, L2 error {e_ref:.6e}")

    res = {}
    for prec in ("fp64", "fp32_refined"):
        if w.u_exact is not None:
            extra, err, st = calibrate(hh, f, g, u_ex, w, prec, e_ref)
            rtol = 0.0
        else:
            # no exact solution: the solve runs to a relative residual of 1e-10 (the stopping
            # rule of the smooth-coefficient workload); err is the distance to the converged
            # float64 solution
            extra, rtol = 100, 1e-10
            u, st = hh.fmg_solve(f, g, nu=w.nu, pre=w.pre, post=w.post, precision=prec, rtol=rtol, max_iter=extra)
            err = l2_error(hh, u, u_ex)
        ms, st, est = timed_steps(hh, f, g, w, prec, extra, args.steps, args.warmup, rtol)
        res[prec] = dict(extra_cycles=st.ir_steps, l2_error=err, ms=ms, vcycles=st.vcycles,
                         dofs_per_s=N / (ms * 1e-3), eta_1=est["eta_j"], theta=est["theta"], dense_level=st.dense_level)
        if rtol:
            res[prec]["rtol"] = rtol
        dense = f"levels 0..{st.dense_level} as a dense map" if st.dense_level >= 1 else "no dense coarse map"
        log(f"{prec}: FMG + {st.ir_steps} extra cycles, L2 error {err:.6e}, {st.vcycles} V-cycles, {ms:.2f} ms/step, "
            f"{N / (ms * 1e-3):.3e} DoF/s, eta_1 {est['eta_j']:.4e}, {dense}")

    sm = {}
    for prec in ("fp64", "fp32_refined"):
        hh.bench_smoother(prec, 2)
        b = hh.bench_smoother(prec, args.sweeps)
        sm[prec] = dict(gbs=b["bytes"] / (b["ms"] * 1e-3) / 1e9, dof_updates_per_s=N * args.sweeps / (b["ms"] * 1e-3),
                        launch_ms=b["launch_ms"], launch_bytes=b["launch_bytes"])
        log(f"smoother {prec}: {sm[prec]['gbs']:.1f} GB/s algorithmic per sweep, "
            f"{sm[prec]['dof_updates_per_s']:.3e} DoF-updates/s, interior launch {b['launch_ms']*1e3:.1f} us")

    k = sm["fp32_refined"]
    achieved = k["launch_bytes"] / (k["launch_ms"] * 1e-3) / 1e9
    kname = KERNEL_NAME.get((w.mesh.dim, w.smoother, w.coefficient), "k_smooth_interior")
    if w.mesh.dim == 3 and 2 ** w.L > 32:
        # 3D levels above n = 32 (the macro does not fit in LDS): red-black with a per-macro
        # coefficient sweeps whole planes at n = 64 and streams tiles from n = 256 on (both
        # colours in one launch), other smoothers and levels go class by class
        rbm = w.smoother == "redblack" and w.coefficient == "macro"
        if rbm and 2 ** w.L >= 256:
            kname = "k_gs3d_stream<float, true>"
        elif rbm and 2 ** w.L == 64:
            kname = "k_gs3d_planes<float, 64, true>"
        else:
            kname = "k_gs3d_rows<float, true>" if 2 ** w.L >= 128 else "k_smooth_interior"
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=TRAFFIC_BYTES.get((w.name, w.L, kname)),
                kernel=kname, bytes_per_launch=k["launch_bytes"], avg_launch_us=round(k["launch_ms"] * 1e3, 2))

    # the whole finest-level sweep (interior and interface) and the whole step against the same
    # peak: algorithmic bytes over measured time
    roof["sweep_frac"] = round(sm["fp32_refined"]["gbs"] / HBM_PEAK_GBS, 4)
    nd = [hh.num_dofs(l) for l in range(w.L + 1)]
    for prec in ("fp64", "fp32_refined"):
        r = res[prec]
        extra = r["vcycles"] - w.nu * w.L
        sb = step_algorithmic_bytes(nd, w.mesh.dim, w.nu, w.pre, w.post, w.nu * w.L, extra, prec, norms="rtol" in r)
        r["step_algorithmic_bytes"] = sb
        r["step_frac"] = round(sb / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    roof["step_frac"] = res["fp32_refined"]["step_frac"]

    ms = res["fp32_refined"]["ms"]
    out = {
        "metric": "FMG DoF/s + smoother HBM GB/s at fixed L2 error; FP32-refined vs FP64",
        "value": round(N / (ms * 1e-3), 1),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 smoothing/transfer inside f64 residual+update (estimator f64)",
        "data": "synthetic",
        "config": {"workload": w.name, "macros": w.mesh.n_cells, "L": w.L, "dofs": N, "smoother": w.smoother,
                   "fmg_nu": w.nu, "vcycle": [w.pre, w.post], "fixed_l2_error": e_ref},
        "fp64": {k2: (float(f"{v:.6g}") if isinstance(v, float) else v) for k2, v in res["fp64"].items()},
        "fp32_refined": {k2: (float(f"{v:.6g}") if isinstance(v, float) else v) for k2, v in res["fp32_refined"].items()},
        "speedup_fp32_refined_vs_fp64": round(res["fp64"]["ms"] / ms, 3),
        "smoother_gbs": {p: round(v["gbs"], 1) for p, v in sm.items()},
        "smoother_dof_updates_per_s": {p: float(f"{v['dof_updates_per_s']:.4e}") for p, v in sm.items()},
        "roofline": roof,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
