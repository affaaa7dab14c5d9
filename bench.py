#!/usr/bin/env python
"""Benchmark of the hot path on one MI355X.

Workload: unit cube, 256^3 interior points, tanh wall stretching (factor 1.5), 8 seeded
non-overlapping spheres, manufactured u = sin(2 pi x) cos(pi y) exp(z), f = (1 - 5 pi^2) u,
g = u.  Inputs are synthetic, generated once and resident in HBM before timing.

One step = the whole hot path on that input: setup (1D coefficients, classification, IBIs,
modified rows, right-hand side), the warm start (when a trained network is available),
and the FP32-inner / FP64-refinement BiCGSTAB solve to ||r||/||b|| <= 1e-10 (and the same
bound on the Jacobi-weighted residual).  The plain FP64 solve of the same problem is timed
once beside it for the speedup; the CPU oracle is timed on a bounded sample.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--parity-tol", type=float, default=1e-13,
                    help="tolerance of the extra solves compared against the stored oracle samples")
    ap.add_argument("--precond", choices=("multigrid", "chebyshev"), default="multigrid",
                    help="inner solver of the K preconditioner (both precisions)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain 1 GiB device copy (HBM reference and counter calibration)")
    ap.add_argument("--workload", choices=("spheres8", "bodies16"), default="spheres8",
                    help="spheres8: the 256^3 benchmark problem; bodies16: the 512^3 scale problem (16 bodies, "
                         "Fourier source, g = 0; no warm start, no oracle samples)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time a full oracle solve of the 128^3 sphere problem on the host (one JSON line)")
    return ap.parse_args()


def cpu_full():
    """The CPU oracle's full FP64 solve (setup + BiCGSTAB to 1e-10, its Chebyshev-Jacobi
    preconditioner) of the 128^3 stretched-grid sphere problem u = exp(x + y + z), timed on
    this host.  The oracle is plain single-threaded C."""
    import numpy as np

    import oracle
    from paper_1901_08269_amd import workloads as W
    w = W.sphere_exp(128)
    t0 = time.perf_counter()
    P = oracle.Problem.from_workload(w)
    t1 = time.perf_counter()
    u, st = P.solve(1e-10)
    t2 = time.perf_counter()
    t = P.types()
    fl = (t == 1) | (t == 2)
    n_unk = int(fl.sum())
    print(json.dumps({"kind": "oracle", "workload": "sphere_exp_128: 128^3 interior, tanh 2.0, sphere r = 0.25, "
                                                    "u = exp(x + y + z), tol 1e-10, Chebyshev-Jacobi preconditioner",
                      "cores": 1, "host_cpus": len(os.sched_getaffinity(0)), "setup_s": t1 - t0, "solve_s": t2 - t1,
                      "total_s": t2 - t0, "iters": st["iters"], "rel_residual": st["rel_residual"],
                      "n_unknowns": n_unk, "unknown_iters_per_s": n_unk * st["iters"] / (t2 - t1),
                      "max_error_vs_exact": float(np.max(np.abs(u - w.u_exact)[fl]))}), flush=True)


def copy_calibration():
    """A plain device-to-device copy of 1 GiB (torch's copy kernel), timed with events: the
    measured HBM copy bandwidth, and the known byte count that FETCH_SIZE / WRITE_SIZE
    counters are scaled against."""
    import torch
    n = 1 << 28   # 2^28 floats = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": ms,
                      "GBps_read_plus_write": 8 * n / (ms * 1e-3) / 1e9}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cpu_full:
        cpu_full()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1901_08269_amd as cps
    from paper_1901_08269_amd import metrics
    from paper_1901_08269_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}), flush=True)
        sys.exit(3)
    t_gen = time.time()
    learned = None
    if args.workload == "bodies16":
        if args.N == 256:
            args.N = 512
        x, _, phi, g, f = W.bodies16_fourier_torch(args.N)
        w = W.Workload(f"bodies16_fourier_{args.N}", x, x, x, None, None, None, meta={"N": args.N})
        dev = {"x": torch.as_tensor(x).cuda(), "y": torch.as_tensor(x).cuda(), "z": torch.as_tensor(x).cuda(),
               "phi": phi, "g": g, "f": f}
        workload = (f"bodies16_fourier_{args.N}: {args.N}^3 interior, tanh 2.0, 8 spheres + 8 ellipsoids seed 1, "
                    f"Fourier f K = 16, g = 0, tol {args.tol:g}")
    else:
        w = W.spheres8(args.N)
        dev = {k: torch.as_tensor(getattr(w, k), dtype=torch.float64).cuda().contiguous()
               for k in ("x", "y", "z", "phi", "g", "f")}
        workload = (f"spheres8_{args.N}: {args.N}^3 interior, tanh 1.5, 8 spheres seed 0, "
                    f"u = sin(2pi x) cos(pi y) exp(z), tol {args.tol:g}")
        try:
            from paper_1901_08269_amd import learned as _learned
            learned = _learned.load_default(args.N) if hasattr(_learned, "load_default") else None
        except Exception as exc:  # the warm start is optional; the plain solve judges
            print(f"# no warm start: {exc}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(f"# inputs generated in {time.time() - t_gen:.1f}s", file=sys.stderr, flush=True)

    side = torch.cuda.Stream()        # the warm start's stream when it runs beside the setup
    # the warm start's launches are made from a worker thread (the library calls release the
    # interpreter lock), so that the setup's host work does not wait behind them
    import concurrent.futures
    launcher = concurrent.futures.ThreadPoolExecutor(max_workers=1)

    def step(precision, timing, precond=None, tol=None, warm=True, overlap=False):
        """setup + (warm start) + solve; returns (u, stats) with the warm start's time in
        stats["predict_ms"] (inference and prolongation, 0 without it).  With overlap the warm
        start is queued on its own stream before the setup and runs beside it; predict_ms is
        then only the time the host waits for it after the setup."""
        use = warm and learned is not None and precision == "mixed"
        u0, pms = None, 0.0
        if use and overlap:
            side.wait_stream(torch.cuda.current_stream())    # the fields, before the setup's work
            fut = launcher.submit(learned.predict_fields, dev["phi"], dev["g"], dev["f"], side, False)
        S = cps.Solver(dev["x"], dev["y"], dev["z"], dev["phi"], dev["g"], dev["f"], precision=precision,
                       kernel_timing=timing, precond=precond or args.precond)
        if use and overlap:
            ta = time.perf_counter()
            u0 = fut.result()
            side.synchronize()
            pms = (time.perf_counter() - ta) * 1e3
        elif use:
            ta = time.perf_counter()
            u0 = learned.predict(S, w)     # returns after the model's stream has synchronised
            pms = (time.perf_counter() - ta) * 1e3
        u, st = S.solve(tol or args.tol, u0=u0, inplace=u0 is not None)
        st["predict_ms"] = pms
        S.close()
        return u, st

    for _ in range(args.warmup):
        step("mixed", False, overlap=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for q in range(args.steps):
        # the full-traffic preconditioner sweeps on the problem's grid in every 8th run of them
        # are timed by events that each sweep's launch stamps with the kernel's own start and
        # end; sweeps queued after convergence are left out
        u, st = step("mixed", 8, overlap=True)
        stats.append(st)
        print(f"# step {q}: {st['iters']} iters, {st['refine_steps']} refinements, "
              f"rel res {st['rel_residual']:.2e}, warm-start wait {st['predict_ms']:.2f} ms, solve {st['solve_ms']:.2f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    last = stats[-1]
    med = lambda v: float(np.median(v))
    solve_s = med([s_["solve_ms"] for s_ in stats]) / 1e3
    # the timed steps run the warm start beside the setup; its own time is measured apart,
    # after the setup, on the solver of one more step
    predict_exposed_s = med([s_["predict_ms"] for s_ in stats]) / 1e3
    predict_s = None
    if learned is not None:
        S_ = cps.Solver(dev["x"], dev["y"], dev["z"], dev["phi"], dev["g"], dev["f"], precision="mixed",
                        precond=args.precond)
        pt = []
        for _ in range(3):
            ta = time.perf_counter()
            learned.predict(S_, w)
            pt.append((time.perf_counter() - ta) * 1e3)
        S_.close()
        predict_s = med(pt) / 1e3
    else:
        predict_s = 0.0
    warm_solve_s = solve_s + predict_s
    t_mask = None
    err = None
    if w.u_exact is not None:
        ue = torch.as_tensor(w.u_exact).cuda()
        _, types = cps.Solver(dev["x"], dev["y"], dev["z"], dev["phi"], dev["g"], dev["f"]).rhs_and_types()
        t_mask = (types == 1) | (types == 2)
        err = float(torch.max(torch.abs(u - ue)[t_mask]))

    # the same mixed solve from a zero start: what the warm start saves
    zero = None
    if learned is not None:
        zs = [step("mixed", False, warm=False)[1] for _ in range(min(args.steps, 3))]
        zero = {"iters": zs[-1]["iters"], "solve_s": med([z["solve_ms"] for z in zs]) / 1e3}
        zero["iters_saved"] = zero["iters"] - last["iters"]
        zero["s_saved_incl_inference"] = zero["solve_s"] - warm_solve_s

    fp64 = None
    if not args.no_fp64:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        u64, st64 = step("fp64", False)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        diff = float(torch.max(torch.abs(u - u64)[t_mask]) / torch.max(torch.abs(u64)[t_mask])) if t_mask is not None else None
        fp64 = {"precond": args.precond, "step_s": tb - ta, "solve_s": st64["solve_ms"] / 1e3,
                "iters": st64["iters"], "rel_residual": st64["rel_residual"], "mixed_vs_fp64_rel_maxdiff": diff}
        if args.steps > 1:
            fp64["solve_s"] = med([st64["solve_ms"]] + [step("fp64", False)[1]["solve_ms"]
                                                        for _ in range(min(args.steps, 3) - 1)]) / 1e3
        if args.precond != "chebyshev":
            # the plain method with the Chebyshev-Jacobi inner solver of K as well
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, stc = step("fp64", False, "chebyshev")
            torch.cuda.synchronize()
            tb = time.perf_counter()
            fp64["chebyshev"] = {"step_s": tb - ta, "solve_s": stc["solve_ms"] / 1e3, "iters": stc["iters"],
                                 "rel_residual": stc["rel_residual"]}

    # parity: both precisions at a tighter tolerance against the stored FP64 oracle samples
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_spheres8_{args.N}.txt")
    if not args.no_fp64 and args.parity_tol > 0:
        parity = {"tol": args.parity_tol}
        samples = None
        if os.path.exists(gold):
            data = np.loadtxt(gold, comments="#")
            umax = [float(l.split()[-1]) for l in open(gold) if l.startswith("# max_abs_u_fluid")][0]
            samples = (torch.as_tensor(data[:, 0].astype(np.int64)).cuda(), torch.as_tensor(data[:, 1]).cuda(), umax)
        for prec in ("mixed", "fp64"):
            up, stp = step(prec, False, tol=args.parity_tol)
            ent = {"solve_s": stp["solve_ms"] / 1e3, "predict_s": stp["predict_ms"] / 1e3, "iters": stp["iters"],
                   "rel_residual": stp["rel_residual"], "rel_residual_jacobi": stp["rel_residual_jacobi"]}
            if samples is not None:
                got = up.reshape(-1)[samples[0]]
                ent["vs_oracle_rel_maxdiff"] = float(torch.max(torch.abs(got - samples[1])) / samples[2])
                ent["oracle_samples"] = int(samples[0].numel())
            parity[prec] = ent
        parity["speedup_mixed_learned_vs_fp64_solve"] = parity["fp64"]["solve_s"] / (
            parity["mixed"]["solve_s"] + parity["mixed"]["predict_s"])
        if samples is not None:
            got = u.reshape(-1)[samples[0]]
            parity["headline_solution_vs_oracle_rel_maxdiff"] = float(torch.max(torch.abs(got - samples[1])) / samples[2])

    # roofline of the dominant kernel, k_cheb4: every Chebyshev sweep of the multigrid smoother
    # on the problem's grid (first steps of a pass: 3 vectors per point; the others: 4), timed
    # live by the library with events that each sweep's launch stamps
    sweeps = sum(s_["sweep_launches"] for s_ in stats)
    sweep_ms = sum(s_["sweep_ms"] for s_ in stats)
    sweep_bytes = sum(s_["sweep_bytes"] for s_ in stats)
    avg_ms = sweep_ms / max(sweeps, 1)
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweeps else None
    full_n = sum(s_["sweep_full_launches"] for s_ in stats)
    full_ms = sum(s_["sweep_full_ms"] for s_ in stats)
    full_bytes = full_n * 4 * 4 * last["sweep_points"]      # the timed steps are the mixed solve's (FP32)
    full_gbs = full_bytes / (full_ms * 1e-3) / 1e9 if full_n else None
    # HBM traffic per launch from the committed counter report, only while it still
    # describes the kernel sources (the report carries their hash) and this workload
    from paper_1901_08269_amd import profiling
    traffic, traffic_note = None, "no counter report for this workload"
    tag = f"{args.workload}_{args.N}"
    rep = profiling.read_traffic(os.path.join(ROOT, "profiles", f"k_cheb4_{tag}_traffic.md"))
    if rep is not None:
        if rep.get("kernel_source_sha256_16") == profiling.source_hash():
            traffic = float(rep["traffic_bytes_per_launch"])
            traffic_note = f"profiles/k_cheb4_{tag}_traffic.md (FETCH_SIZE+WRITE_SIZE, copy-calibrated)"
        else:
            traffic_note = "kernel sources changed since the counters were taken"
    roofline = {"kernel": "k_cheb4<float, *> (every smoother sweep on the problem's grid: first steps of a pass "
                          "<float, true, 2> and the others <float, false, 1>; per-launch averages)",
                "bound": "hbm", "achieved": achieved, "peak": metrics.MI355X_HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / metrics.MI355X_HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_source": traffic_note,
                "avg_launch_us": avg_ms * 1e3, "launches": sweeps,
                "bytes_per_launch": sweep_bytes / max(sweeps, 1),
                "full_sweeps_only": {"kernel": "k_cheb4<float, false, 1>", "launches": full_n,
                                     "avg_launch_us": full_ms * 1e3 / max(full_n, 1), "achieved": full_gbs,
                                     "frac": (full_gbs / metrics.MI355X_HBM_PEAK_GBS) if full_gbs else None}}

    cpu = None
    if not args.no_cpu_baseline and args.workload == "spheres8":
        # the oracle's preconditioner is the Chebyshev-Jacobi inner solve: scale to the iteration
        # count of the GPU FP64 solve with that preconditioner (the GPU parity tests hold the two
        # counts within a few iterations of each other)
        if fp64 and "chebyshev" in fp64:
            cheb_iters = fp64["chebyshev"]["iters"]
        elif fp64 and args.precond == "chebyshev":
            cheb_iters = fp64["iters"]
        else:
            cheb_iters = last["iters"]
        cpu = cpu_baseline(w, args, cheb_iters)

    opts = cps.default_options()
    setup_s = med([s_["setup_ms"] for s_ in stats]) / 1e3
    n_unk = last["n_unknowns"]
    out = {
        "metric": "solve s to 1e-10 rel residual at 256^3 (mixed+learned vs FP64); stencil GB/s",
        "value": ms_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": workload,
                   "precision": "mixed", "warm_start": "learned" if learned is not None else "zero",
                   "precond": args.precond,
                   "precond_settings": ({"levels": opts.mg_levels, "nu": opts.mg_nu,
                                         "coarse_steps": opts.mg_coarse_steps,
                                         "smooth_interval": [opts.mg_smooth_lo, opts.lam_hi]}
                                        if args.precond == "multigrid" else
                                        {"inner_iters": opts.inner_iters,
                                         "cheb_interval": [max(opts.lam_hi / (4.0 * opts.inner_iters ** 2),
                                                               (1 - np.cos(np.pi / (args.N + 1)))), opts.lam_hi]})},
        "solve_s": solve_s,
        "predict_s": predict_s,
        # the part of the warm start that the timed steps waited for after the setup (it is
        # queued on its own stream before the setup and runs beside it)
        "predict_exposed_s": predict_exposed_s,
        "solve_incl_inference_s": warm_solve_s,
        "setup_s": setup_s,
        "iters": last["iters"],
        "iters_fp32": last["iters_fp32"],
        "refine_steps": last["refine_steps"],
        "rel_residual": last["rel_residual"],
        "rel_residual_jacobi": last["rel_residual_jacobi"],
        "max_error_vs_exact": err,
        "n_unknowns": n_unk,
        "n_irregular": last["n_irregular"],
        "unknown_iters_per_s": n_unk * last["iters"] / solve_s,
        "unknown_iters_per_s_fp32_inner": n_unk * last["iters_fp32"] / solve_s,
        "zero_start": zero,
        "fp64": fp64,
        # plain FP64 solve from zero against the mixed solve with its warm start's inference
        # and prolongation included (setup excluded on both sides); medians over the steps
        "speedup_vs_fp64_solve": (fp64["solve_s"] / warm_solve_s) if fp64 else None,
        "speedup_vs_fp64_solve_excl_inference": (fp64["solve_s"] / solve_s) if fp64 else None,
        "speedup_vs_fp64_chebyshev_solve": (fp64["chebyshev"]["solve_s"] / warm_solve_s)
        if fp64 and "chebyshev" in fp64 else None,
        "parity": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(w, args, iters_full):
    """The CPU oracle, timed on the same workload: its setup plus `cpu_iters` FP64 BiCGSTAB
    iterations (Chebyshev-Jacobi preconditioner), scaled to `iters_full` iterations, the count
    of the GPU FP64 solve with the same preconditioner (seconds per solve)."""
    import oracle
    t0 = time.perf_counter()
    P = oracle.Problem.from_workload(w)
    t1 = time.perf_counter()
    _, st = P.solve(args.tol, max_iters=args.cpu_iters, check=False)
    t2 = time.perf_counter()
    per_iter = (t2 - t1) / max(st["iters"], 1)
    return {"value": (t1 - t0) + per_iter * iters_full, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup + {st['iters']} FP64 BiCGSTAB iteration(s) on the same {args.N}^3 workload "
                      f"({t2 - t0:.1f}s of CPU work), scaled to {iters_full} iterations (the GPU FP64 solve's count "
                      f"with the oracle's Chebyshev-Jacobi preconditioner)",
            "setup_s": t1 - t0, "iter_s": per_iter}


if __name__ == "__main__":
    main()
