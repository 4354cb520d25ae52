"""Benchmark: gradient evaluations per second on the 256 x 256 x 128 workload.

One step = one full gradient evaluation (forward convolution on the cells the
objective reads, J in FP64, adjoint convolution onto the design cells,
dJ/drho) through the C ABI, with rho already resident in HBM.

Prints one JSON line: the FP32 rate (the value), the plain FP64 GPU rate and
their ratio, the dominant kernel against the HBM roofline (per-launch HIP
events on the launch stream, algorithmic bytes from the pass sizes), and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gradient evals/s (fwd+adjoint) at 256x256x128 FP32 vs FP64 plain; HBM GB/s"
HBM_PEAK_GBS = 8000.0
# rocprofv3 summary of this workload (kernel trace + FETCH_SIZE / WRITE_SIZE runs)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "gradient_eval_256x256x128_kernels.md")


def model_bytes_per_eval(w, wsize, L):
    """Full-field pass model of one gradient evaluation (two scalar
    convolutions over the whole padded box, zero padding never stored, the
    tensor spectrum octant read once per convolution)."""
    nx, ny, nz = w.n
    Lx, Ly, Lz = L
    hx = Lx // 2 + 1
    per_field = nx * ny * nz + 4 * hx * ny * nz + 4 * hx * Ly * nz
    K = hx * (Ly // 2 + 1) * (Lz // 2 + 1)
    return wsize * (2 * 2 * per_field + 2 * K + nx * ny * nz)


def time_steps(torch, e, rho, grad, J, steps):
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        e.objective_and_grad(rho, grad, J)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def cpu_baseline(w, layers=16):
    """The oracle (direct sums, FP64) on the host cores: the full forward
    field on the objective's cells, J and dJ/dH, and the adjoint on `layers`
    of the design layers; the adjoint time is scaled to all design layers
    (its cost is linear in the number of target cells)."""
    import oracle
    table = oracle.table_for(w)        # setup, not timed
    t0 = time.perf_counter()
    H = oracle.forward_field(w, table=table)
    J, g = oracle.objective(w, H)
    t1 = time.perf_counter()
    x0, x1, y0, y1, z0, z1 = w.design
    sub = (x0, x1, y0, y1, z1 - layers, z1)
    A = oracle.field(w.n, w.h, g, oracle.objective_box(w), sub, oracle.objective_mask(w),
                     oracle.m0_mask(w), table)
    oracle.gradient_from_adjoint(w, A)
    t2 = time.perf_counter()
    per_eval = (t1 - t0) + (t2 - t1) * (z1 - z0) / layers
    return {"value": 1.0 / per_eval, "unit": "gradient evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one evaluation: full forward direct sum on the {w.sensor[1]-w.sensor[0]+2}x"
                      f"{w.sensor[3]-w.sensor[2]+2} objective cells, adjoint direct sum on {layers} of "
                      f"{z1 - z0} design layers scaled linearly; FP64; {t2 - t0:.1f} s measured"}


def batch_measurement(torch, wl, args):
    """64 independent designs of uneven size (FP32), schedules (padded
    lengths and pass structure) chosen by the autotuner, one graph replay per
    batch evaluation."""
    from paper_1707_09898_amd import autotune
    from paper_1707_09898_amd.batch import DesignBatch
    ws = wl.config5()
    t0 = time.perf_counter()
    lengths = passes = None
    if not args.no_autotune:
        sched = [autotune.tune_schedule(w, "f32", evals=2)[0] for w in ws]
        lengths = [L for L, _ in sched]
        passes = [name for _, name in sched]
    t1 = time.perf_counter()
    b = DesignBatch(ws, "f32", lengths, streams=args.batch_streams, passes=passes)
    nbytes = b.algorithmic_bytes()
    b.capture()
    for _ in range(3):
        b.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.batch_replays):
        b.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.batch_replays
    # eager launches of the same batch, for comparison
    b.run_eager()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        b.run_eager()
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / 5
    cells = int(sum(int(w.n[0]) * int(w.n[1]) * int(w.n[2]) for w in ws))
    res = {"designs": len(ws), "cells": cells, "ms_per_batch": ms, "evals_per_s": len(ws) * 1000.0 / ms,
           "ms_per_batch_eager": ms_eager, "bytes_per_batch": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9,
           "streams": args.batch_streams, "autotuned": not args.no_autotune,
           "autotune_s": round(t1 - t0, 1),
           "lengths": [list(map(int, e.padded_lengths())) for e in b.engines],
           "passes": passes}
    b.close()
    print(f"[bench] c5 batch: {ms:.3f} ms per 64 designs ({res['evals_per_s']:.0f} evals/s), eager {ms_eager:.3f} ms",
          file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--f64-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-design batch measurement")
    ap.add_argument("--no-paths", action="store_true", help="skip timing the unfused pass choices")
    ap.add_argument("--batch-replays", type=int, default=20)
    ap.add_argument("--batch-streams", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true", help="batch with the default padded lengths")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB three times (a known-size kernel for "
                         "calibrating memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1707_09898_amd import tof, workloads as wl

    torch.cuda.set_device(0)
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copied {args.calibrate_copy_mib} MiB x3", file=sys.stderr, flush=True)
        del a, b
    w = wl.config3()
    print(f"[bench] workload {w.name}, steps {args.steps}, warmup {args.warmup}", file=sys.stderr, flush=True)

    results = {}
    for dtype, steps in (("f32", args.steps), ("f64", args.f64_steps)):
        e = tof.engine_for(w, dtype)
        L = e.padded_lengths()
        rho = torch.as_tensor(w.rho, dtype=e.dtype, device="cuda")
        grad = torch.empty_like(rho)
        J = torch.empty(1, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            e.objective_and_grad(rho, grad, J)
        ms = time_steps(torch, e, rho, grad, J, steps)
        J_main = float(J.item())
        grad_main = grad.double()   # the timed path's gradient, for the precision report
        # per-launch timing in a second pass over the same number of steps
        e.profile(True)
        for _ in range(args.profile_steps):
            e.objective_and_grad(rho, grad, J)
        prof = e.profile_read()
        kernels = e.profile_kernels(with_items=True)
        e.profile(False)
        paths = {}
        if dtype == "f32" and not args.no_paths:
            # the same evaluation on the other pass choices (direct z sum unfused; FFTs along z)
            for name, (zs, fu, fo) in (("zsum", (1, 0, 0)), ("zfft", (0, 0, 0))):
                e.set_option(tof.OPT_ZSUM, zs)
                e.set_option(tof.OPT_FUSE_YZ, fu)
                e.set_option(tof.OPT_FUSE_OBJECTIVE, fo)
                for _ in range(3):
                    e.objective_and_grad(rho, grad, J)
                paths[name] = 1000.0 / time_steps(torch, e, rho, grad, J, max(10, steps // 4))
            for opt in (tof.OPT_ZSUM, tof.OPT_FUSE_YZ, tof.OPT_FUSE_OBJECTIVE):
                e.set_option(opt, 1)
        results[dtype] = {"ms": ms, "prof": prof, "kernels": kernels, "L": L, "J": J_main, "paths": paths}
        print(f"[bench] {dtype}: {ms:.4f} ms/eval, {1000.0 / ms:.1f} evals/s, J={J_main:.10e}",
              file=sys.stderr, flush=True)
        results[dtype]["grad"] = grad_main
        e.close()
        del rho, grad

    r32 = results["f32"]
    wsize = 4
    evals = 1000.0 / r32["ms"]
    slots = [(name, ms_tot / cnt, cnt, by) for (name, ms_tot, cnt, by) in r32["prof"] if cnt > 0]
    dom = max(slots, key=lambda s: s[1])
    dom_idx = tof.PROFILE_NAMES.index(dom[0])
    dom_kernel, dom_items = r32["kernels"][dom_idx]
    achieved = dom[3] / (dom[1] * 1e-3) / 1e9
    from paper_1707_09898_amd import rocprof_summary
    traffic, same_src = rocprof_summary.lookup(TRAFFIC_SUMMARY, dom_kernel, "float", dom_items)
    traffic_note = ("FETCH_SIZE + WRITE_SIZE bytes per launch (copy-calibrated), "
                    + os.path.relpath(TRAFFIC_SUMMARY, ROOT)) if traffic is not None and same_src else \
        ("kernel sources changed since the counters were taken" if traffic is not None else
         ("no counter summary for this kernel launch" if os.path.exists(TRAFFIC_SUMMARY) else
          "counter summary file not found: " + os.path.relpath(TRAFFIC_SUMMARY, ROOT)))
    if not same_src:
        traffic = None
    pass_bytes = sum(by for (_, _, cnt, by) in slots)
    model = model_bytes_per_eval(w, wsize, r32["L"])
    out = {
        "metric": METRIC,
        "value": evals,
        "unit": "gradient evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded rho ~ U[0,1], p=3, M0=(0,0,1))",
        "config": {"workload": "c3: 256x256x128 cubic cells padded 512x512x256, design z<124, "
                               "64x64 sensor plane at z=127, J=mean(Hz-0.2)^2+0.01 mean|grad_xy Hz|^2",
                   "global_batch": 1, "parallelism": "single GPU"},
        "f64_plain": {"value": 1000.0 / results["f64"]["ms"], "ms_per_step": results["f64"]["ms"],
                      "steps": args.f64_steps},
        "speedup_f32_over_f64": results["f64"]["ms"] / r32["ms"],
        # FP32 against the plain FP64 path on the same input (the FP64 path
        # itself is pinned to the oracle at 1e-10 by the parity tests)
        "precision_f32_vs_f64": {
            "J_rel": abs(r32["J"] - results["f64"]["J"]) / abs(results["f64"]["J"]),
            "grad_rel_inf": float((r32["grad"] - results["f64"]["grad"]).abs().max() /
                                  results["f64"]["grad"].abs().max())},
        "bytes_per_eval": {"passes": pass_bytes, "full_field_model": model},
        "effective_GBps": {"passes": pass_bytes * evals / 1e9, "full_field_model": model * evals / 1e9},
        "per_kernel_us": {f"{name}:{r32['kernels'][tof.PROFILE_NAMES.index(name)][0]}": round(avg * 1e3, 2)
                          for (name, avg, _, _) in slots},
        "paths_f32_evals_per_s": dict({"fused": evals}, **r32["paths"]),
        "roofline": {"bound": "hbm", "kernel": f"{dom_kernel} ({dom[0]}, {dom_items} work items)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_note": traffic_note,
                     "bytes_per_launch": dom[3], "avg_launch_us": dom[1] * 1e3},
    }
    if not args.no_batch:
        out["c5_batch"] = batch_measurement(torch, wl, args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
