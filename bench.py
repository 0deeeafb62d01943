"""Benchmark: lambda-sweep PCG solves per second on one MI355X.

Workload (the 512 x 512 deblurring configuration): 15 x 15 Gaussian PSF
(sigma = 3) with reflective boundary, Neumann gradient, seeded
piecewise-constant phantom with 1% noise, three outer weightings
(D = I, then seeded edge weights in [0.01, 1]) and 20 lambdas log-spaced in
[1e-5, 1]; a six-level V-cycle preconditioner.  One step = for every outer
weighting: install the weights (Galerkin hierarchy) and solve the whole
lambda sweep to relative residual 4e-13, a tolerance at which every
solution is within relative error 1e-6 of the FP64 oracle (checked by the
GPU test suite at this size and setting).  Each weighting's sweep starts from the
previous weighting's solutions (warm start across outer iterations).
60 solves per step, FP64 throughout.

Prints one JSON line.  `value` = solves / second of the timed steps with the
inputs resident in HBM.  `roofline` reports the most frequent kernel (the
finest-level Chebyshev smoothing step) from HIP events around every run of
its consecutive launches in a second pass over the same step.  `mixed_fp32`
times the same step once more with the V-cycle in FP32 under flexible FP64
PCG (same tolerance; its solutions meet the same 1e-6 bar in the GPU test
suite) and reports its speedup over the FP64 step.  `cpu_baseline` times
the CPU oracle on a bounded sample (see its `sample` field).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TOL = 4e-13
NU_FINE, RATIO_FINE = 128, 3.0e5
NU_COARSE, RATIO_COARSE = 2, 4.0
CT_TOL = 1e-12
HBM_PEAK_GBS = 8000.0
COPY_PROBE_BYTES = 256 << 20    # calibration copy for the traffic counters


def workload_config(P_):
    return {
        "workload": (f"deblur {P_.nv}x{P_.nh}, 15x15 Gaussian PSF sigma=3, "
                     "reflective blur, Neumann gradient, 3 outer weightings x "
                     f"{len(P_.lams)} lambdas in [1e-5, 1], {P_.levels}-level "
                     f"V-cycle (Chebyshev nu={NU_FINE} fine / {NU_COARSE} "
                     f"coarse), rel. residual {TOL:g} (rel. error <= 1e-6)"),
        "n": P_.nv * P_.nh,
        "lambdas": len(P_.lams),
        "outer": len(P_.weights),
        "solves_per_step": len(P_.lams) * len(P_.weights),
    }


def run_step(prob, b, D, lams, bufs):
    """One step: the outer weightings in order, each sweep started from the
    previous weighting's solutions (zero for the first)."""
    infos = []
    x0 = None
    for k, d in enumerate(D):
        prob.set_weights(d)
        x, _, _, info = prob.solve_sweep(b, lams, TOL, x0=x0, x=bufs[k & 1],
                                         maxit=400000, poll_every=16)
        x0 = x
        infos.append(info)
    return infos


def traffic_per_launch(n, launches, nbytes):
    """HBM traffic per k_smooth_fine launch for the live launch mix, from the
    committed FETCH_SIZE / WRITE_SIZE counters (two launch sizes, scaled by
    a plain copy's counts), or None when the kernel's sources have changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_smooth_fine_traffic.json")
    if not os.path.exists(path) or launches == 0:
        return None
    with open(path) as fh:
        J = json.load(fh)
    h = hashlib.sha256()
    for src in J["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != J["sources_sha256"] or J["n"] != n:
        return None
    pts = sorted(J["points"], key=lambda p: p["slots"])
    t = [1024.0 * (p["fetch_kib"] * J["fetch_scale"] +
                   p["write_kib"] * J["write_scale"]) for p in pts]
    z = [p["slots"] for p in pts]
    slope = (t[-1] - t[0]) / (z[-1] - z[0])
    icpt = t[0] - slope * z[0]
    # the timer's bytes are n (32 z + 16) summed over launches (three-term
    # form of the tiled FP64 step)
    slot_launches = (nbytes / n - 16.0 * launches) / 32.0
    return (icpt * launches + slope * slot_launches) / launches


def cpu_baseline(P_, iters_per_slot, budget_s=20.0):
    """Time the oracle's V-cycle-preconditioned CG on the same workload for a
    bounded number of iterations and extrapolate with the per-lambda
    iteration counts of the GPU run (the two agree to +-1 iteration)."""
    import numpy as np

    from oracle.pcg import DeblurOracle, pcg

    O = DeblurOracle(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                     P_.weights[1], P_.levels)
    lam = float(P_.lams[0])
    nus = [NU_FINE] + [NU_COARSE] * (P_.levels - 1)
    ratios = [RATIO_FINE] + [RATIO_COARSE] * (P_.levels - 1)
    t_setup0 = time.perf_counter()
    c0 = time.process_time()
    V = O.vcycle(lam, nu=nus, ratio=ratios)
    K = O.K(lam)
    f = O.rhs(P_.b)
    t_setup = time.perf_counter() - t_setup0
    # one iteration to size the sample, then one bounded run
    t1 = time.perf_counter()
    pcg(K, f, V, tol=0.0, maxit=1)
    one = time.perf_counter() - t1
    total_its = max(2, int(budget_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    pcg(K, f, V, tol=0.0, maxit=total_its)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    per_it = wall / total_its
    total_slot_its = float(np.sum(iters_per_slot))
    solves = len(iters_per_slot)
    est = total_slot_its * per_it
    return {
        "value": solves / est,
        "unit": "solves/s",
        "cores": max(1, round(cpu / (wall + t_setup))),
        "kind": "oracle",
        "sample": (f"{total_its} MG-PCG iterations of the CPU oracle (numpy/"
                   f"scipy FP64) at lambda={lam:g}, outer weighting 1, "
                   f"{wall:.1f} s; time per iteration {per_it:.3f} s "
                   f"extrapolated to the {int(total_slot_its)} iterations the "
                   f"{solves} solves of one step take"),
    }


def run_ct(args):
    """The tomography sweep: every weighting warm-started from the previous
    one, relative residual CT_TOL, the benchmark's smoothing."""
    import numpy as np
    import torch

    from paper_2306_11067_amd import TomographyProblem
    from workloads.ct import config3

    P = config3()
    dev = torch.device("cuda:0")
    b = torch.as_tensor(P.b).to(dev)
    D = [torch.as_tensor(w).to(dev) for w in P.weights]
    lams = np.asarray(P.lams)
    prob = TomographyProblem(P.rowptr, P.col, P.val, P.N, P.levels,
                             nu=NU_FINE, cheb_ratio=RATIO_FINE, weights=D[0],
                             nu_coarse=NU_COARSE,
                             cheb_ratio_coarse=RATIO_COARSE)
    bufs = [torch.empty(len(lams) * P.n, dtype=torch.float64, device=dev)
            for _ in range(2)]
    prob.solve_sweep(b, lams, CT_TOL, maxit=2, poll_every=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos, x0 = [], None
        for k, d in enumerate(D):
            prob.set_weights(d)
            x, _, _, info = prob.solve_sweep(b, lams, CT_TOL, x0=x0,
                                             x=bufs[k & 1], maxit=400000,
                                             poll_every=16)
            x0 = x
            infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solves = args.steps * len(lams) * len(D)
    iters = [i["iters"] for info in infos for i in info]
    out = {
        "metric": "lambda-sweep PCG solves/sec (tomography workload)",
        "value": solves / elapsed, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 0,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic (seeded ellipse phantom, exact-length projector)",
        "config": {"workload": (f"CT {P.N}x{P.N} parallel beam, "
                                f"{P.n_angles} angles x {P.n_bins} bins, "
                                f"nnz {int(P.rowptr[-1])}, {len(P.weights)} "
                                f"weightings x {len(lams)} lambdas in "
                                f"[1e-3, 1e2], {P.levels} levels, Chebyshev "
                                f"nu={NU_FINE}, rel. residual {CT_TOL:g}"),
                   "max_iterations": max(iters),
                   "all_converged": all(i["flags"] & 1 for info in infos
                                        for i in info)},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


OUTER_Q = 2.0      # exponent of the weight update (the paper leaves it open)
OUTER_MAX = 12


def outer_loop(prob, b, lams):
    """One timed call of the library's Algorithm 2 from D = I."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, chosen, info = prob.regularize(b, lams, OUTER_Q, TOL,
                                      maxouter=OUTER_MAX, poll_every=16)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = len(lams) + 10 * (info["outer"] - 1)
    return {"wall_s": dt, "outer": info["outer"], "stopped": info["stopped"],
            "chosen": chosen, "solves": solves, "solves_per_s": solves / dt,
            "pcg_iterations": info["iters"], "q": OUTER_Q}


def run_outer(prob, b, lams, P_):
    """Algorithm 2 on the 512 x 512 workload: one timed call of the
    library's outer loop (sweeps, corner choices, weight updates)."""
    o = outer_loop(prob, b, lams)
    print(json.dumps({
        "metric": "Algorithm 2 wall time (outer reweighting loop)",
        "value": o["wall_s"], "unit": "s", "higher_is_better": False,
        "n_gpus": 1, "dtype": "f64",
        "data": "synthetic (seeded phantom, PSF, noise)",
        "outer_iterations": o["outer"], "stopped": o["stopped"],
        "chosen": o["chosen"], "solves": o["solves"],
        "solves_per_s": o["solves_per_s"], "pcg_iterations": o["pcg_iterations"],
        "q": OUTER_Q,
        "config": {"workload": "deblur 512x512, 15x15 Gaussian PSF sigma=3, "
                               "reflective blur, Neumann gradient, 20 lambdas "
                               "in [1e-5, 1], D = I at the start, pruned "
                               "sweeps of 10 lambdas after the first, "
                               f"rel. residual {TOL}"}}), flush=True)


def run_paper_deblur(n):
    """Algorithm 2 on the deblurring problem of the paper's Section 4.6
    (zero-boundary anisotropic Toeplitz blur, 30 lambdas in [1e-3, 1e2])."""
    import torch
    import workloads as W
    from paper_2306_11067_amd import Problem
    P_ = W.paper_deblur(n)
    b = torch.as_tensor(P_.b).cuda()
    prob = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels, nu=NU_FINE, cheb_ratio=RATIO_FINE,
                   nu_coarse=NU_COARSE, cheb_ratio_coarse=RATIO_COARSE)
    prob.solve_sweep(b, P_.lams, TOL, maxit=2, poll_every=2)
    o = outer_loop(prob, b, P_.lams)
    prob.close()
    print(json.dumps({
        "metric": "Algorithm 2 wall time (outer reweighting loop)",
        "value": o["wall_s"], "unit": "s", "higher_is_better": False,
        "n_gpus": 1, "dtype": "f64",
        "data": "synthetic (seeded shapes phantom, 1% noise)",
        "outer_iterations": o["outer"], "stopped": o["stopped"],
        "chosen": o["chosen"], "solves": o["solves"],
        "solves_per_s": o["solves_per_s"], "pcg_iterations": o["pcg_iterations"],
        "q": OUTER_Q,
        "config": {"workload": f"paper deblurring {n}x{n}: zero-boundary "
                               "Toeplitz blur, Gaussians radius 6 sigma "
                               f"{1.25 * n / 64:g} / radius 7 sigma "
                               f"{1.5 * n / 64:g}, Neumann gradient, 30 "
                               "lambdas in [1e-3, 1e2], "
                               f"{P_.levels}-level V-cycle, rel. residual "
                               f"{TOL}"}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workload", default="deblur512",
                    choices=["deblur512", "ct256", "paper_deblur256"],
                    help="ct256: the 256x256 parallel-beam tomography sweep "
                         "(32 lambdas, 2 weightings, FP32 V-cycle under FP64 "
                         "PCG); prints its own JSON line without roofline")
    ap.add_argument("--no-outer", action="store_true")
    ap.add_argument("--outer", action="store_true",
                    help="run Algorithm 2 (outer reweighting loop with L-curve "
                         "choice, pruning and stopping rule) on the 512x512 "
                         "workload from D = I; prints its own JSON line")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the launches the HBM traffic counters are "
                         "taken on (a copy of known size, then 4 iterations "
                         "at 20 and at 1 lambda with direct launches)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the "
              "lambda sweep is solved on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2306_11067_amd import Problem

    if args.workload == "ct256":
        return run_ct(args)
    if args.workload == "paper_deblur256":
        return run_paper_deblur(256)

    P_ = W.config2()
    dev = torch.device("cuda:0")
    b = torch.as_tensor(P_.b).to(dev)
    D = [torch.as_tensor(w).to(dev) for w in P_.weights]
    lams = np.asarray(P_.lams)
    prob = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels, nu=NU_FINE, cheb_ratio=RATIO_FINE, weights=D[0],
                   nu_coarse=NU_COARSE, cheb_ratio_coarse=RATIO_COARSE)
    bufs = [torch.empty(len(lams) * P_.nv * P_.nh, dtype=torch.float64,
                        device=dev) for _ in range(2)]
    if args.traffic_probe:
        src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        for lm in (lams, lams[:1]):
            prob.solve_sweep(b, lm, 1e-30, maxit=4, poll_every=2, graph=False)
        torch.cuda.synchronize()
        print("traffic probe done", flush=True)
        return
    # load every kernel once (not a step)
    prob.solve_sweep(b, lams, TOL, maxit=2, poll_every=2)
    if args.outer:
        return run_outer(prob, b, lams, P_)
    for _ in range(args.warmup):
        run_step(prob, b, D, lams, bufs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos = run_step(prob, b, D, lams, bufs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solves = args.steps * len(lams) * len(D)
    conv = all(i["flags"] & 1 for info in infos for i in info)
    iters = [i["iters"] for info in infos for i in info]
    print(f"timed {args.steps} step(s) in {elapsed:.2f} s, all converged: "
          f"{conv}, max iterations {max(iters)}", file=sys.stderr, flush=True)

    roof = None
    if not args.no_roofline:
        # the same step again, kernels launched one by one, each run of
        # consecutive dominant-kernel launches bracketed by HIP events
        prob.kernel_timer(True)
        run_step(prob, b, D, lams, bufs)
        torch.cuda.synchronize()
        launches, seconds, nbytes = prob.kernel_timer_read()
        prob.kernel_timer(False)
        avg_s = seconds / max(launches, 1)
        achieved = (nbytes / max(launches, 1)) / avg_s / 1e9
        tr = traffic_per_launch(P_.nv * P_.nh, launches, nbytes)
        roof = {"bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if tr is None else round(tr),
                "kernel": "k_smooth_fine (finest-level Chebyshev step)",
                "launches": launches,
                "avg_launch_us": round(1e6 * avg_s, 3),
                "bytes_per_launch": round(nbytes / max(launches, 1))}
        print(f"roofline pass: {launches} launches, {1e6 * avg_s:.2f} us "
              f"avg, {achieved:.1f} GB/s", file=sys.stderr, flush=True)

    mixed = None
    if not args.no_mixed:
        # the same step with the FP32 V-cycle under flexible FP64 PCG
        prob32 = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                         P_.levels, nu=NU_FINE, cheb_ratio=RATIO_FINE,
                         weights=D[0], nu_coarse=NU_COARSE,
                         cheb_ratio_coarse=RATIO_COARSE,
                         precision="mixed_fp32")
        prob32.solve_sweep(b, lams, TOL, maxit=2, poll_every=2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        inf32 = run_step(prob32, b, D, lams, bufs)
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t1
        conv32 = all(i["flags"] & 1 for info in inf32 for i in info)
        it32 = [i["iters"] for info in inf32 for i in info]
        prob32.close()
        mixed = {"value": len(lams) * len(D) / el32, "unit": "solves/s",
                 "ms_per_step": 1e3 * el32,
                 "speedup_vs_fp64": (elapsed / args.steps) / el32,
                 "all_converged": conv32, "max_iterations": max(it32),
                 "arithmetic": "FP32 V-cycle (vectors, bands, stencils), "
                               "FP64 PCG vectors, dots, residual, tail"}
        print(f"mixed step in {el32:.2f} s (speedup "
              f"{mixed['speedup_vs_fp64']:.2f}), all converged: {conv32}, "
              f"max iterations {max(it32)}", file=sys.stderr, flush=True)

    outer = None
    if not args.no_outer:
        # Algorithm 2 on the same workload (the outer loop around sweeps);
        # reported beside the step, not part of it
        outer = outer_loop(prob, b, lams)
        print(f"outer loop: {outer['wall_s']:.2f} s, {outer['outer']} outer "
              f"iterations, chosen {outer['chosen']}", file=sys.stderr,
              flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P_, iters)

    out = {
        "metric": ("lambda-sweep PCG solves/sec at rel.err 1e-6 vs FP64 "
                   "oracle; % HBM roofline"),
        "value": solves / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded phantom, PSF, noise and edge weights)",
        "config": workload_config(P_),
        "roofline": roof,
        "cpu_baseline": cpu,
        "mixed_fp32": mixed,
        "outer_loop": outer,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
