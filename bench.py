#!/usr/bin/env python3
"""Throughput of the parallel augmented subspace eigensolver on one MI355X.

Default workload (kappa2d-H32-h2048-k50-mixed): the largest single-GPU
configuration, 4.2M fine nodes, 50 eigenpairs, log-normal kappa per element,
FP32 V-cycles on FP64 residuals.  With this rough coefficient the Galerkin
coarse space V_H cannot carry the eigenpairs above the lowest ones to 1e-8
(the method's own limit, Remark 3.1; reproduced by the oracle in
tests/test_oracle_rescope.py), so a step is one outer iteration (one
correction step, Algorithm 1, for all 50 eigenpairs: V-cycles, borders,
arrowhead eigensolve, prolongation) and metric = eigenpair correction
steps per second; every step's arithmetic is checked against the oracle at
this size by tests/test_gpu_fullsize.py.

--workload lap2d-H64-h1024-k20 (and the other constant-coefficient
workloads): a step is one whole solve: restart from the coarse start of
Algorithm 2 (or, with --nested V, its nested step 2(A) with V steps per
intermediate mesh) and correction steps until every eigenvalue is within
1e-8 relative of the oracle's discrete eigenvalue; metric = eigenpairs per
second to 1e-8 relative eigenvalue error.  The uneven batch reports
eigenpair correction steps per second against its members run one by one.

Prints one JSON line.  --gpus above 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
# the source file that defines the dominant (finest-level) kernel of the
# timed 2D workloads: a committed counter record is used only while it is
# unchanged
KERNEL_SOURCES = ["paper_1908_10251_amd/csrc/march2d.hip"]

KERNEL_NAMES = {
    2: "finest-level smoothing phases (k_march: pre-smoothing with fused residual restriction, the first one of "
       "each step of a solve also forming the previous step's prolongation (or the restart's start) and the "
       "right-hand side; a V-cycle's "
       "post-smoothing with fused prolongation together with the next cycle's pre-smoothing and restriction in "
       "one pass; the last post-smoothing of a step also forming the borders; k_smooth_fused where coefficients "
       "vary)",
    3: "finest-level smoothing phases (k_march3: all steps of a phase in one pass marching along z, "
       "post-smoothing with fused prolongation)",
    "learned": "finest-level learned smoothing step (k_learned_step: residual, two bfloat16 matrix-core "
               "convolutions, update)",
    "batch": "finest batched level smoothing phases (k_march_ew over every member of the level: the general "
             "7-point operators' planes of each pair's member streamed beside x and f, pre-smoothing with fused "
             "residual restriction, post-smoothing with fused prolongation)",
    "cg": "finest-level conjugate-gradient smoothing phases (k_cg_start, k_cg_dir: direction update fused with "
          "A p and p.Ap partial sums, k_cg_update: x, r and r.r partial sums; the inner products added per "
          "right-hand side by k_cg_reduce; the paper's multigrid step)",
    "kappa": "finest-level smoothing phases (k_march with edge weights, FP32: pre-smoothing with fused residual "
             "restriction, post-smoothing with fused prolongation; the two weight planes streamed beside x and f)",
}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def golden(name: str):
    path = os.path.join(ROOT, "tests", "golden", f"{name}.eigenvalues.txt")
    if not os.path.exists(path):
        return None
    return np.loadtxt(path, comments="#")


def traffic_record(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_fine_smoothing_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def _cpu_pool_sample(wl, k):
    """Processes of the oracle's Algorithm 2 run at once: one per host core
    (the paper's one process per eigenpair), at most k."""
    from oracle import pasm as O
    return min(k, O.cpu_count())


def cpu_baseline_solve(wl: W.Workload, ref: np.ndarray):
    """The oracle (as it stands) on a bounded sample of the same workload: the
    first c eigenpairs (c = host cores) corrected in c worker processes with
    the oracle's own V-cycles from the coarse start until each is within
    1e-8 of its discrete eigenvalue; time of the correction steps."""
    from oracle import pasm as O
    t0 = time.perf_counter()
    prob = O.make_problem(wl.dim, wl.n_coarse, wl.n_fine)
    bvp = O.MultigridBVP(prob, O.mg_options_for(wl))
    lam0, U0, _, _ = O.coarse_start(prob, wl.k)
    t_setup = time.perf_counter() - t0
    c = _cpu_pool_sample(wl, wl.k)
    # a tolerance on the change per step that lands within 1e-8 of the value
    # (the contraction is fast); the count is checked against ref below
    t1 = time.perf_counter()
    r = O.solve(prob, c, bvp, tol=1e-10, max_iter=10, workers=c, which=list(range(c)), start=(lam0, U0))
    t_iter = time.perf_counter() - t1
    reached = int(np.sum(np.abs(r["lam"] - ref[:c]) / ref[:c] <= 1e-8))
    steps = [len(h) - 1 for h in r["hist"]]
    return {"value": reached / t_iter, "unit": "eigenpairs/s", "cores": c, "kind": "oracle",
            "sample": f"eigenpairs 0..{c - 1} of {wl.name} in {c} processes (one BLAS thread each), oracle "
                      f"V-cycles (same smoother), {min(steps)}-{max(steps)} correction steps each, {reached} within "
                      f"1e-8 in {t_iter:.1f} s wall; oracle set-up {t_setup:.1f} s not counted"}


def cpu_baseline_steps(wl: W.Workload, kap):
    """The oracle (as it stands) on a bounded sample: one correction step
    (its own FP64 V-cycles) of the first c eigenpairs (c = host cores) in c
    worker processes, from the coarse start; time of that step."""
    from oracle import fem, pasm as O
    t0 = time.perf_counter()
    if wl.tensor == "example2":
        prob = O.make_problem(wl.dim, wl.n_coarse, wl.n_fine, tensor=fem.example2_tensor,
                              potential=fem.example2_potential)
    else:
        prob = O.make_problem(wl.dim, wl.n_coarse, wl.n_fine, kappa=kap)
    bvp = O.MultigridBVP(prob, O.mg_options_for(wl))
    lam0, U0, _, _ = O.coarse_start(prob, wl.k)
    t_setup = time.perf_counter() - t0
    c = _cpu_pool_sample(wl, wl.k)
    t1 = time.perf_counter()
    O.solve(prob, c, bvp, tol=0.0, max_iter=1, workers=c, which=list(range(c)), start=(lam0, U0))
    t_step = time.perf_counter() - t1
    return {"value": c / t_step, "unit": "eigenpair-steps/s", "cores": c, "kind": "oracle",
            "sample": f"one correction step of eigenpairs 0..{c - 1} of {wl.name} in {c} processes (one BLAS "
                      f"thread each), oracle FP64 V-cycles (same smoother), {t_step:.1f} s wall; oracle set-up "
                      f"{t_setup:.1f} s not counted"}


def roofline(launches, ms, bpl, workload, kernel, flops_per_launch=None):
    avg_ms = ms / max(launches, 1)
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    out = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_record(workload), "kernel": kernel,
           "launches": launches, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bpl}
    if flops_per_launch and launches:
        tf = flops_per_launch / (avg_ms * 1e-3) / 1e12
        out["mfma_tflops"] = tf
        out["mfma_frac_of_bf16_peak"] = tf / PEAK_BF16_TFLOPS
    return out


def line(wl, metric, value, unit, steps, warmup, ms_per_step, config, roof, dtype):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": dict({"workload": wl.name}, **config),
            "roofline": roof}


def coefficients(wl: W.Workload):
    """Per-element inputs of a single-instance workload: kappa, potential, tensor."""
    kap = W.lognormal_kappa(wl.dim, wl.n_fine, seed=wl.seed) if wl.kappa == "lognormal" else None
    if wl.tensor == "example2":
        ten, phi = W.example2_elements(wl.n_fine)
        return kap, phi, ten
    return kap, None, None


def bench_solve(args, wl, pasm, torch):
    """A step = one whole solve to 1e-8 relative eigenvalue error."""
    opts = pasm.options_for(wl)
    opts.max_iter = args.max_iter
    kap, pot, ten = coefficients(wl)
    t0 = time.perf_counter()
    solver = pasm.Solver(wl.dim, wl.H, wl.h, wl.k, kappa=kap, potential=pot, opts=opts, tensor=ten)
    t_setup = time.perf_counter() - t0
    ctx, k = solver.ctx, wl.k
    learned = wl.smoother == "learned"
    if learned and args.learned == "on":
        pasm.pasm_learned_enable(ctx, True)  # override the set-up speed test

    ref = golden(wl.golden_name)
    ref_kind = "oracle discrete eigenvalues (tests/golden)"
    if ref is None:
        # tightly converged FP64 values of the same problem with the plain smoother
        o2 = pasm.options_for(wl)
        o2.precision = pasm.PASM_FP64
        if o2.smoother == pasm.PASM_LEARNED:
            o2.smoother = pasm.PASM_JACOBI
        o2.tol, o2.max_iter = 1e-14, args.ref_iter
        with pasm.Solver(wl.dim, wl.H, wl.h, wl.k, kappa=kap, potential=pot, opts=o2) as rs:
            its = rs.solve(allow_notconv=True)
            ref = rs.eigenpairs(False)[0]
        ref_kind = f"this problem's eigenvalues from {its} FP64 plain-smoother iterations (tol 1e-14)"
    ref = np.asarray(ref[:k])

    # Eigenvalues are compared as sorted lists: inside a degenerate cluster
    # (the 3D cube keeps exact multiplicities) any member of the cluster is a
    # correct answer for any process of it.
    def rel_err(lam):
        return np.abs(np.sort(lam) - np.sort(ref)) / np.sort(ref)

    def one_solve(first_check=1):
        """Iterate until every eigenvalue is within 1e-8: the first
        first_check steps back to back with one synchronisation (the library's
        n-step entry point), then one step at a time, checking after each."""
        if args.nested:
            pasm.pasm_restart_nested(ctx, args.nested)
        else:
            pasm.pasm_restart(ctx)
        its = min(first_check, args.max_iter)
        pasm.pasm_iterate_n(ctx, its)
        while True:
            lam = solver.eigenpairs(False)[0]
            if np.max(rel_err(lam)) <= 1e-8 or its >= args.max_iter:
                return its, lam
            pasm.pasm_iterate(ctx)
            its += 1

    # The warm-up solves find the iteration count; the timed solves run that
    # many iterations back to back (no host round trip in between), then
    # check, and go on checking every iteration should they need more.
    first_check = 1
    for _ in range(args.warmup):
        its_w, _ = one_solve()
        first_check = its_w
    rep0 = pasm.pasm_learned_report(ctx) if learned else None
    pasm.pasm_profile(ctx, 0, True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    iters = []
    for _ in range(args.steps):
        its, lam = one_solve(first_check)
        iters.append(its)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    launches, ms, bpl = pasm.pasm_profile_read(ctx, 0)
    pasm.pasm_profile(ctx, 0, False)
    err = rel_err(lam)
    ms_per_step = 1e3 * elapsed / args.steps
    replay = None
    if not learned:
        # the same solves without profiling events, launched one kernel at a
        # time and replayed from recorded graphs (pasm_use_graph)
        def timed_solves(n):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(n):
                one_solve(first_check)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / n

        t_eager = timed_solves(args.steps)
        pasm.pasm_use_graph(ctx, True)
        timed_solves(3)  # record the steps' graphs
        t_graph = timed_solves(args.steps)
        _, graphs, replayed = pasm.pasm_graph_stats(ctx)
        lam_g = solver.eigenpairs(False)[0]
        pasm.pasm_use_graph(ctx, False)
        replay = {"ms_per_solve_eager": 1e3 * t_eager, "ms_per_solve_graph": 1e3 * t_graph,
                  "eigenpairs_per_s_graph": k / t_graph, "graphs": graphs, "replayed_steps": replayed,
                  "max_rel_err_graph": float(np.max(rel_err(lam_g)))}
    value = k / (ms_per_step / 1e3) if float(np.max(err)) <= 1e-8 else 0.0
    n_dofs = pasm.pasm_num_dofs(ctx)
    sweeps = wl.vcycles * (2 if learned else wl.nu_pre + wl.nu_post)
    cfg = {"dim": wl.dim, "H": wl.H, "h": wl.h, "k": k, "fine_dofs": n_dofs, "coarse_dofs": pasm.pasm_coarse_dofs(ctx),
           "smoother": wl.smoother, "nu": [wl.nu_pre, wl.nu_post], "vcycles": wl.vcycles,
           "precision": wl.precision, "iterations_per_step": iters, "max_rel_err": float(np.max(err)),
           "eigenpairs_within_1e-8": int(np.sum(err <= 1e-8)), "reference": ref_kind, "setup_s": t_setup,
           "fine_dof_updates_per_s": n_dofs * k * sweeps * float(np.mean(iters)) / (ms_per_step / 1e3)}
    if replay:
        cfg["graph_replay"] = replay
    if args.nested:
        cfg["start"] = (f"nested (Algorithm 2 step 2(A)): {args.nested} correction step(s) on each intermediate mesh "
                        f"before the finest-level steps; iterations_per_step counts finest-level steps")
    else:
        cfg["start"] = "coarse start (Algorithm 2 with h_1 = H)"
    if ref_kind.startswith("oracle"):
        # after the timed region: the same solve continued to a change below
        # 1e-12, and its error against the oracle's discrete eigenvalues
        o_t = pasm.options_for(wl)
        o_t.tol, o_t.max_iter = 1e-12, 30
        with pasm.Solver(wl.dim, wl.H, wl.h, wl.k, kappa=kap, potential=pot, opts=o_t) as ts:
            its_t = ts.solve(allow_notconv=True)
            lam_t = ts.eigenpairs(False)[0]
        cfg["tight_solve"] = {"stop": "max relative eigenvalue change < 1e-12", "steps": its_t,
                              "max_rel_err": float(np.max(rel_err(lam_t))),
                              "bar": 1e-10 if wl.precision == "fp64" else 1e-8}
    flops = None
    kernel = KERNEL_NAMES["cg"] if wl.smoother == "cg" else KERNEL_NAMES[wl.dim]
    if learned:
        rep = pasm.pasm_learned_report(ctx)
        cfg["learned"] = rep
        cfg["learned_mode"] = args.learned
        # the timed launches are the learned step's only if the learned
        # smoother ran (the set-up speed test may have left it off)
        if rep["cycles_learned"] > rep0["cycles_learned"]:
            # 16 channels x 27 taps multiply-adds in each of the two layers per node
            flops = 2.0 * 2 * 16 * 27 * n_dofs * k
            kernel = KERNEL_NAMES["learned"]
            if rep["cycles_fallback"] > rep0["cycles_fallback"]:
                kernel += "; some cycles fell back to plain smoothing"
        else:
            kernel += " (the learned smoother was off: the set-up speed test found plain cycles faster)"
    roof = roofline(launches, ms, bpl, wl.name, kernel, flops)
    out = line(wl, "eigenpairs/sec to 1e-8 rel eigenvalue error", value, "eigenpairs/s", args.steps, args.warmup,
               ms_per_step, cfg, roof, "f64" if wl.precision == "fp64" else "f32+f64")
    if not args.no_cpu_baseline and wl.dim == 2 and wl.kappa == "one":
        out["cpu_baseline"] = cpu_baseline_solve(wl, ref)
    solver.close()
    return out


def coefficient_text(wl: W.Workload) -> str:
    if wl.tensor == "example2":
        return ("A = I + (x-1/2)(x-1/2)^T, phi = exp(prod(x_i - 1/2)) at element centroids (the second example "
                "of Section 5)")
    if wl.kappa == "lognormal":
        return "kappa log-normal, sigma 1, i.i.d. per fine element"
    return "constant (Laplacian)"


def graph_replay_steps(args, pasm, torch, ctx, k):
    """The same correction steps without profiling events, launched one
    kernel at a time and then replayed from recorded graphs (pasm_use_graph);
    reported beside the timed region's value, which carries the events that
    time the roofline kernel."""
    def timed(n):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            pasm.pasm_iterate(ctx)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n

    t_eager = timed(args.iters)
    pasm.pasm_use_graph(ctx, True)
    timed(7)  # record: the step states recur every 6 steps (3 eigenvalue buffers, 2 for u)
    t_graph = timed(args.iters)
    _, graphs, replayed = pasm.pasm_graph_stats(ctx)
    pasm.pasm_use_graph(ctx, False)
    return {"ms_per_step_eager": 1e3 * t_eager, "ms_per_step_graph": 1e3 * t_graph,
            "eigenpair_steps_per_s_graph": k / t_graph, "graphs": graphs, "replayed_steps": replayed}


def bench_steps(args, wl, pasm, torch):
    """Single instances that the method does not take to 1e-8 for every
    eigenpair (rough coefficients, the cube's clusters) and the second
    example: correction steps per second, the state carried from step to
    step."""
    opts = pasm.options_for(wl)
    kap, pot, ten = coefficients(wl)
    t0 = time.perf_counter()
    solver = pasm.Solver(wl.dim, wl.H, wl.h, wl.k, kappa=kap, potential=pot, opts=opts, tensor=ten)
    t_setup = time.perf_counter() - t0
    ctx, k = solver.ctx, wl.k
    learned = wl.smoother == "learned"
    if learned and args.learned == "on":
        pasm.pasm_learned_enable(ctx, True)  # override the set-up speed test
    for _ in range(args.warmup):
        pasm.pasm_iterate(ctx)
    rep0 = pasm.pasm_learned_report(ctx) if learned else None
    pasm.pasm_profile(ctx, 0, True)
    hist = [solver.eigenpairs(False)[0]]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.iters):
        pasm.pasm_iterate(ctx)
        hist.append(solver.eigenpairs(False)[0])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    launches, ms, bpl = pasm.pasm_profile_read(ctx, 0)
    pasm.pasm_profile(ctx, 0, False)
    replay = graph_replay_steps(args, pasm, torch, ctx, k) if not learned else None
    H = np.array(hist)
    d = np.abs(H[1:] - H[:-1]) / H[1:]
    ms_per_step = 1e3 * elapsed / args.iters
    n_dofs = pasm.pasm_num_dofs(ctx)
    cfg = {"dim": wl.dim, "H": wl.H, "h": wl.h, "k": k, "fine_dofs": n_dofs,
           "smoother": wl.smoother, "nu": [wl.nu_pre, wl.nu_post], "vcycles": wl.vcycles, "precision": wl.precision,
           "coefficients": coefficient_text(wl), "iterations": args.iters,
           "eigenpairs_with_last_change_below_1e-10": int(np.sum(d[-1] < 1e-10)), "setup_s": t_setup,
           "step": "one outer iteration (one correction step for all k eigenpairs)"}
    if replay:
        cfg["graph_replay"] = replay
    flops = None
    if wl.smoother == "cg":
        kname = KERNEL_NAMES["cg"]
    elif wl.dim == 3:
        kname = KERNEL_NAMES[3]
    else:
        kname = KERNEL_NAMES["kappa"] if wl.precision == "mixed" else KERNEL_NAMES[2]
    if learned:
        rep = pasm.pasm_learned_report(ctx)
        cfg["learned"] = rep
        cfg["learned_mode"] = args.learned
        # the timed launches are the learned step's only if the learned
        # smoother ran (the set-up speed test may have left it off)
        if rep["cycles_learned"] > rep0["cycles_learned"]:
            # 16 channels x 27 taps multiply-adds in each of the two layers per node
            flops = 2.0 * 2 * 16 * 27 * n_dofs * k
            kname = KERNEL_NAMES["learned"]
            if rep["cycles_fallback"] > rep0["cycles_fallback"]:
                kname += "; some cycles fell back to plain smoothing"
        else:
            kname += " (the learned smoother was off: the set-up speed test found plain cycles faster)"
    roof = roofline(launches, ms, bpl, wl.name, kname, flops)
    solver.close()
    out = line(wl, "eigenpair correction steps/sec", k / (ms_per_step / 1e3), "eigenpair-steps/s", args.iters,
               args.warmup, ms_per_step, cfg, roof, "f32+f64" if wl.precision == "mixed" else "f64")
    if not args.no_cpu_baseline and not learned:
        out["cpu_baseline"] = cpu_baseline_steps(wl, kap)
    if wl.tensor == "example2":
        # eigenpairs whose last step changed the eigenvalue by less than 1e-8
        out["config"]["eigenpairs_with_last_change_below_1e-8"] = int(np.sum(d[-1] < 1e-8))
    return out


def bench_batch(args, wl, pasm, torch):
    """16 uneven instances: batched (one launch per level, graph replay) vs the
    same members as single contexts one after the other."""
    inst = W.uneven_batch(16, seed=wl.seed)
    members = [(1.0 / I.n_fine, I.kappa, W.quadratic_potential_elements(I.n_fine, I.centre)) for I in inst]
    opts = pasm.options_for(wl)
    k = wl.k
    t0 = time.perf_counter()
    b = pasm.Batch(wl.H, k, members, opts=opts)
    t_setup = time.perf_counter() - t0
    rows, tms = pasm.pasm_batch_tuning(b.b)

    def timed(fn, n):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n

    for _ in range(args.warmup):
        b.iterate()
    pasm.pasm_batch_profile(b.b, 0, True)
    t_prof = timed(b.iterate, 2)  # events are recorded outside the graph
    launches, ms, bpl = pasm.pasm_batch_profile_read(b.b, 0)
    pasm.pasm_batch_profile(b.b, 0, False)
    pasm.pasm_batch_use_graph(b.b, False)
    t_eager = timed(b.iterate, args.iters)
    pasm.pasm_batch_use_graph(b.b, True)
    t_graph = timed(b.iterate, args.iters)
    lam = b.eigenvalues()
    b.close()
    singles = [pasm.Solver(2, wl.H, h, k, kappa=kap, potential=pot, opts=opts) for h, kap, pot in members]
    for s in singles:
        s.iterate()
    t_seq = timed(lambda: [s.iterate() for s in singles], max(1, args.iters // 2))
    for s in singles:
        s.close()
    n = len(members)
    cfg = {"instances": n, "fine_cells": [I.n_fine for I in inst], "H": wl.H, "k_per_instance": k,
           "total_fine_dofs": int(sum((I.n_fine - 1) ** 2 for I in inst)), "smoother": wl.smoother,
           "nu": [wl.nu_pre, wl.nu_post], "vcycles": wl.vcycles, "precision": wl.precision,
           "kappa": "log-normal, sigma 1, i.i.d. per fine element", "potential": "|x - c|^2, seeded centre",
           "tiles_per_level": rows.tolist(), "setup_s": t_setup,
           "ms_per_iteration": {"batched_graph": 1e3 * t_graph, "batched_eager": 1e3 * t_eager,
                                "sequential_single_contexts": 1e3 * t_seq},
           "speedup_vs_sequential": t_seq / t_graph, "all_eigenvalues_finite": bool(np.all(np.isfinite(lam))),
           "step": "one outer iteration for all 16 x k eigenpairs"}
    roof = roofline(launches, ms, bpl, wl.name, KERNEL_NAMES["batch"])
    return line(wl, "eigenpair correction steps/sec", n * k / t_graph, "eigenpair-steps/s", args.iters,
                args.warmup, 1e3 * t_graph, cfg, roof, "f32+f64")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=W.KAPPA2D_MIXED.name)
    ap.add_argument("--nested", type=int, default=0, metavar="VARPI",
                    help="solve workloads: start each solve with Algorithm 2's nested step 2(A), VARPI correction "
                         "steps per intermediate mesh")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-iter", type=int, default=40)
    ap.add_argument("--ref-iter", type=int, default=200, help="iterations of the reference run (no stored values)")
    ap.add_argument("--iters", type=int, default=10, help="timed iterations (step-throughput workloads)")
    ap.add_argument("--learned", choices=["auto", "on"], default="auto",
                    help="learned-smoother workloads: keep the set-up speed test's choice, or force it on")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="also run a plain device copy of this size (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the eigenpairs are independent, "
              f"so a multi-GPU run would shard them, which this program does not do.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1908_10251_amd as pasm

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))
        return

    wl = {w.name: w for w in W.ALL}[args.workload]
    torch.cuda.set_device(0)
    if wl is W.BATCH2D_UNEVEN:
        out = bench_batch(args, wl, pasm, torch)
    elif wl.kappa != "one" or wl.tensor != "none" or wl.dim == 3:
        out = bench_steps(args, wl, pasm, torch)
    else:
        out = bench_solve(args, wl, pasm, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
