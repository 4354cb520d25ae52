"""Benchmark: gradient evaluations per second on the 256 x 256 x 128 workload.

One step = one full gradient evaluation (forward convolution on the cells the
objective reads, J in FP64, adjoint convolution onto the design cells,
dJ/drho) through the C ABI, with rho already resident in HBM.  The timed
path is the sensor-pruned one (x transforms, then the y transforms fused
with a direct sum along z against the x-y transformed tensor, since the
objective reads one z layer); its own byte model is the sum of the passes'
algorithmic bytes.  The five-pass FFT pipeline (FFTs along all three axes,
the tensor product per frequency) is measured beside it, as the field of the
whole grid and as the gradient, against the full-field byte model.

Prints one JSON line: the FP32 rate (the value: the median of 5 timed loops
of K steps each), the plain FP64 GPU rate and their ratio, the dominant
kernel and the whole evaluation against the HBM roofline (per-launch HIP
events on the launch stream, algorithmic bytes from the pass sizes), the
full-field pipeline, the 64-design batch, and the CPU oracle timed on whole
evaluations of the same workload.
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


def per_field_words(w, L):
    """Words one axis sweep of the five-pass pipeline moves per field: rho or
    the output (n), the x-pass output written and read (4 hx ny nz), the
    y-pass output written and read (4 hx Ly nz)."""
    nx, ny, nz = w.n
    Lx, Ly, Lz = L
    hx = Lx // 2 + 1
    return nx * ny * nz + 4 * hx * ny * nz + 4 * hx * Ly * nz


def spectrum_words(L):
    Lx, Ly, Lz = L
    return (Lx // 2 + 1) * (Ly // 2 + 1) * (Lz // 2 + 1)


def model_bytes_per_eval(w, wsize, L):
    """Full-field pass model of one gradient evaluation (two scalar
    convolutions over the whole padded box, zero padding never stored, the
    tensor spectrum octant read once per convolution)."""
    nx, ny, nz = w.n
    return wsize * (2 * 2 * per_field_words(w, L) + 2 * spectrum_words(L) + nx * ny * nz)


def model_bytes_per_field(w, wsize, L):
    """The same model for one field H_z = -N (*) M (one scalar convolution)."""
    return wsize * (2 * per_field_words(w, L) + spectrum_words(L))


def timed_loops(torch, fn, steps, repeats):
    """ms per call of fn over `repeats` timed loops of exactly `steps` calls,
    each bracketed by device synchronizations (HIP events on the current stream)."""
    out = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        out.append(t0.elapsed_time(t1) / steps)
    return out


def median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, repeats):
    """The oracle (direct sums, FP64, OpenMP over the host cores) on whole
    evaluations of the workload: the forward field on the objective's cells,
    J and dJ/dH, the adjoint on every design cell and dJ/drho; the tensor
    table is setup and not timed.  The median over `repeats` evaluations."""
    import oracle
    table = oracle.table_for(w)        # setup, not timed
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle.objective_and_grad(w, table=table)
        times.append(time.perf_counter() - t0)
        print(f"[bench] oracle evaluation {times[-1]:.2f} s", file=sys.stderr, flush=True)
    per_eval = median(times)
    return {"value": 1.0 / per_eval, "unit": "gradient evals/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "seconds_per_eval": times,
            "sample": f"{repeats} whole evaluations of the same workload (forward direct sum on the "
                      f"{w.sensor[1]-w.sensor[0]+2}x{w.sensor[3]-w.sensor[2]+2} objective cells, adjoint "
                      f"direct sum on all {w.design[5] - w.design[4]} design layers), FP64; median"}


def slot_times(tof, e, call, steps, burst_launches, bursts):
    """Per-slot timing of engine e's calls: `steps` calls with an event per
    launch (prof: per slot (name, total ms, launches, bytes per launch);
    kernels: per slot (kernel name, work items)), then `bursts` calls in which
    every slot's pass is launched again `burst_launches` times back to back
    with HIP events around the burst only (an event bound to each launch
    lengthens it); burst_ms per slot: the median of the bursts' mean ms per
    launch, 0.0 where no burst ran (no bursts asked for, or a pass that works
    in place)."""
    e.profile(True)
    for _ in range(steps):
        call()
    prof = e.profile_read()
    kernels = e.profile_kernels(with_items=True)
    active = [i for i, (_, _, cnt, _) in enumerate(prof) if cnt > 0]
    runs = []
    for _ in range(bursts if burst_launches > 0 else 0):
        e.profile_burst(active, burst_launches)
        call()
        runs.append(e.profile_burst_read())
    e.profile_read()   # the per-launch records of the burst calls are not used
    e.profile(False)
    burst_ms = [median([r[i] for r in runs]) if runs else 0.0 for i in range(tof.PROFILE_SLOTS)]
    return prof, kernels, burst_ms


def stream_reference(torch, mib=1024, loops=10):
    """What plain streaming kernels reach on this GPU, per read : write mix
    (torch's elementwise kernels over arrays of `mib` MiB of FP32; bytes =
    what each must read and write; median of 3 timed loops): the practical
    ceiling the passes' own read : write mixes can be set against."""
    n = mib * 2 ** 20 // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    c = torch.empty(n, dtype=torch.complex64, device="cuda")
    c.copy_(x)
    cases = {
        "write only (fill)": (lambda: y.fill_(0.5), 4 * n),
        "read 1 : write 2 (real to complex)": (lambda: c.copy_(x), 12 * n),
        "read 1 : write 1 (copy)": (lambda: y.copy_(x), 8 * n),
        "read 2 : write 1 (complex to real part)": (lambda: y.copy_(c.real), 12 * n),
        "read only (sum)": (lambda: x.sum(), 4 * n),
    }
    out = {}
    for name, (fn, by) in cases.items():
        for _ in range(3):
            fn()
        ms = median(timed_loops(torch, fn, loops, 3))
        out[name] = round(by / (ms * 1e-3) / 1e9, 1)
    del x, y, c
    return out


def full_field_measurement(torch, tof, w, steps, repeats, burst_launches=100, bursts=5):
    """The five-pass FFT pipeline at 256 x 256 x 128 FP32: (a) the field H_z
    of the whole grid (tof_field, FFTs along x, y and z with the tensor
    product per frequency), and (b) the gradient with FFTs along z (the
    direct z sums switched off), each against the full-field byte model,
    with the dominant kernel of the field against the HBM roofline."""
    e = tof.engine_for(w, "f32")
    L = e.padded_lengths()
    rho = torch.as_tensor(w.rho, dtype=torch.float32, device="cuda")
    H = torch.empty((1,) + rho.shape, dtype=torch.float32, device="cuda")
    for _ in range(3):
        e.field(rho, comps=4, out=H)
    ms = median(timed_loops(torch, lambda: e.field(rho, comps=4, out=H), steps, repeats))
    prof, kernels, burst_ms = slot_times(tof, e, lambda: e.field(rho, comps=4, out=H), steps, burst_launches, bursts)
    # mean launch time: the burst's, or with an event per launch for a pass that works in place
    slots = [(i, name, burst_ms[i] or t / c, c, by) for i, (name, t, c, by) in enumerate(prof) if c > 0]
    pass_bytes = sum(by for (_, _, _, _, by) in slots)
    dom = max(slots, key=lambda s: s[2])
    model_f = model_bytes_per_field(w, 4, L)
    field = {"what": "tof_field, Hz on all 256x256x128 cells from the 124 design layers (five passes: x R2C, "
                     "y FFT, z FFT + tensor product + inverse z, inverse y, inverse x C2R)",
             "ms_per_field": ms, "fields_per_s": 1000.0 / ms,
             "model_bytes": model_f, "model_GBps": model_f / (ms * 1e-3) / 1e9,
             "model_frac": model_f / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "pass_bytes": pass_bytes, "pass_GBps": pass_bytes / (ms * 1e-3) / 1e9,
             "pass_frac": pass_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "per_kernel_us": {f"{name}:{kernels[i][0]}": round(avg * 1e3, 2) for (i, name, avg, _, _) in slots},
             "per_kernel_timing": {f"{name}:{kernels[i][0]}": ("burst" if burst_ms[i] else "event per launch")
                                   for (i, name, _, _, _) in slots},
             "dominant_kernel": {"kernel": kernels[dom[0]][0], "slot": dom[1], "avg_launch_us": dom[2] * 1e3,
                                 "bytes_per_launch": dom[4],
                                 "achieved_GBps": dom[4] / (dom[2] * 1e-3) / 1e9,
                                 "frac": dom[4] / (dom[2] * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    # the gradient through the same pipeline (z FFTs instead of the direct sums)
    grad = torch.empty_like(rho)
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    for opt in (tof.OPT_ZSUM, tof.OPT_FUSE_YZ):
        e.set_option(opt, 0)
    for _ in range(3):
        e.objective_and_grad(rho, grad, J)
    msg = median(timed_loops(torch, lambda: e.objective_and_grad(rho, grad, J), steps, repeats))
    e.profile(True)
    for _ in range(steps):
        e.objective_and_grad(rho, grad, J)
    prof = e.profile_read()
    e.profile(False)
    gbytes = sum(by for (_, _, c, by) in prof if c > 0)
    model_g = model_bytes_per_eval(w, 4, L)
    gradient = {"what": "tof_objective_and_grad with FFTs along z (direct z sums off)",
                "ms_per_eval": msg, "evals_per_s": 1000.0 / msg,
                "model_bytes": model_g, "model_GBps": model_g / (msg * 1e-3) / 1e9,
                "model_frac": model_g / (msg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "pass_bytes": gbytes, "pass_GBps": gbytes / (msg * 1e-3) / 1e9,
                "pass_frac": gbytes / (msg * 1e-3) / 1e9 / HBM_PEAK_GBS}
    e.close()
    print(f"[bench] full-field pipeline: field {ms:.4f} ms ({field['model_frac']:.2f} of peak on the model), "
          f"gradient {msg:.4f} ms ({gradient['model_frac']:.2f})", file=sys.stderr, flush=True)
    return {"field": field, "gradient": gradient}


def time_batch(torch, b, replays):
    """ms per batch evaluation: median of 3 timed loops of graph replays,
    and the same batch launched eagerly."""
    b.capture()
    for _ in range(3):
        b.replay()
    ms = median(timed_loops(torch, b.replay, replays, 3))
    b.run_eager()
    ms_eager = median(timed_loops(torch, b.run_eager, 5, 3))
    return ms, ms_eager


def batch_measurement(torch, wl, args):
    """64 independent designs of uneven size (FP32).  The batched form: one
    launch per pass and kernel instantiation over device tables of the
    designs (power-of-two padded lengths along x and y), one graph replay per
    batch evaluation.  For comparison, the designs' own launches spread over
    streams in one graph, with schedules (padded lengths and pass structure)
    chosen by the autotuner."""
    from paper_1707_09898_amd import autotune
    from paper_1707_09898_amd.batch import DesignBatch
    ws = wl.config5()
    cells = int(sum(int(w.n[0]) * int(w.n[1]) * int(w.n[2]) for w in ws))
    b = DesignBatch(ws, "f32", mode="batched")
    t0 = time.perf_counter()
    untuned_ms = b.time_eager()
    table, tuned_ms, trials = autotune.tune_batch(b)
    t1 = time.perf_counter()
    nbytes = b.algorithmic_bytes()
    launches = b.launches()
    lengths = [list(map(int, e.padded_lengths())) for e in b.engines]
    ms, ms_eager = time_batch(torch, b, args.batch_replays)
    b.close()
    res = {"designs": len(ws), "cells": cells, "form": "batched launches (tof_batch), one graph",
           "launches_per_batch": launches, "ms_per_batch": ms, "evals_per_s": len(ws) * 1000.0 / ms,
           "ms_per_batch_eager": ms_eager, "bytes_per_batch": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9,
           "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "lengths": lengths,
           "tile_knobs": {k: {str(L): v for L, v in d.items()} for k, d in table.items()},
           "ms_eager_before_tuning": untuned_ms, "tune_s": round(t1 - t0, 1), "tune_trials": len(trials)}
    print(f"[bench] c5 batched: {ms:.3f} ms per 64 designs ({res['evals_per_s']:.0f} evals/s, {launches} launches), "
          f"eager {ms_eager:.3f} ms", file=sys.stderr, flush=True)
    if not args.no_streams_batch:
        t0 = time.perf_counter()
        sched = [autotune.tune_schedule(w, "f32", evals=2)[0] for w in ws]
        t1 = time.perf_counter()
        b = DesignBatch(ws, "f32", [L for L, _ in sched], streams=args.batch_streams, passes=[p for _, p in sched],
                        mode="streams")
        sbytes = b.algorithmic_bytes()
        sms, sms_eager = time_batch(torch, b, args.batch_replays)
        b.close()
        res["streams_form"] = {"form": f"each design's own launches over {args.batch_streams} streams, one graph",
                               "launches_per_batch": 5 * len(ws), "ms_per_batch": sms,
                               "evals_per_s": len(ws) * 1000.0 / sms, "ms_per_batch_eager": sms_eager,
                               "bytes_per_batch": sbytes, "GBps": sbytes / (sms * 1e-3) / 1e9,
                               "autotune_s": round(t1 - t0, 1), "lengths": [list(L) for L, _ in sched],
                               "passes": [p for _, p in sched]}
        print(f"[bench] c5 streams: {sms:.3f} ms per 64 designs", file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--f64-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=3, help="whole oracle evaluations timed (median)")
    ap.add_argument("--repeats", type=int, default=5, help="timed loops of --steps steps (median)")
    ap.add_argument("--no-full-field", action="store_true", help="skip the five-pass pipeline measurement")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--burst-launches", type=int, default=100,
                    help="launches per burst of each pass for the per-kernel times (0: an event per launch)")
    ap.add_argument("--bursts", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-design batch measurement")
    ap.add_argument("--no-stream-reference", action="store_true",
                    help="skip the plain streaming kernels (practical bandwidth per read : write mix)")
    ap.add_argument("--no-paths", action="store_true", help="skip timing the unfused pass choices")
    ap.add_argument("--batch-replays", type=int, default=20)
    ap.add_argument("--batch-streams", type=int, default=4)
    ap.add_argument("--no-streams-batch", action="store_true",
                    help="skip the comparison batch of per-design launches over streams")
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
        loops = timed_loops(torch, lambda: e.objective_and_grad(rho, grad, J), steps, args.repeats)
        ms = median(loops)
        J_main = float(J.item())
        grad_main = grad.double()   # the timed path's gradient, for the precision report
        # bursts for the FP32 value only: FP64 arrays are twice the size, and
        # a pass repeated on its own finds more of its inputs in the chip's
        # last-level cache than it does inside the evaluation
        prof, kernels, burst_ms = slot_times(tof, e, lambda: e.objective_and_grad(rho, grad, J),
                                             args.profile_steps, args.burst_launches if dtype == "f32" else 0,
                                             args.bursts)
        paths = {}
        if dtype == "f32" and not args.no_paths:
            # the same evaluation on the other pass choices (direct z sum unfused; FFTs along z)
            for name, (zs, fu, fo) in (("zsum", (1, 0, 0)), ("zfft", (0, 0, 0))):
                e.set_option(tof.OPT_ZSUM, zs)
                e.set_option(tof.OPT_FUSE_YZ, fu)
                e.set_option(tof.OPT_FUSE_OBJECTIVE, fo)
                for _ in range(3):
                    e.objective_and_grad(rho, grad, J)
                paths[name] = 1000.0 / median(timed_loops(torch, lambda: e.objective_and_grad(rho, grad, J),
                                                          max(10, steps // 4), 3))
            for opt in (tof.OPT_ZSUM, tof.OPT_FUSE_YZ, tof.OPT_FUSE_OBJECTIVE):
                e.set_option(opt, 1)
        results[dtype] = {"ms": ms, "loops": loops, "prof": prof, "kernels": kernels, "L": L, "J": J_main,
                          "paths": paths, "burst_ms": burst_ms}
        print(f"[bench] {dtype}: {ms:.4f} ms/eval, {1000.0 / ms:.1f} evals/s, J={J_main:.10e}",
              file=sys.stderr, flush=True)
        results[dtype]["grad"] = grad_main
        e.close()
        del rho, grad

    r32 = results["f32"]
    wsize = 4
    evals = 1000.0 / r32["ms"]
    # per slot: (name, mean ms per launch, launches, algorithmic bytes per launch, ms with an event per launch);
    # the mean launch time is the burst's where bursts ran
    slots = [(name, r32["burst_ms"][i] or ms_tot / cnt, cnt, by, ms_tot / cnt)
             for i, (name, ms_tot, cnt, by) in enumerate(r32["prof"]) if cnt > 0]
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
    pass_bytes = sum(s[3] for s in slots)
    model = model_bytes_per_eval(w, wsize, r32["L"])
    # measured traffic of the whole evaluation: every timed kernel's counters
    measured = 0.0
    for (name, avg, cnt, by, _) in slots:
        kname, items = r32["kernels"][tof.PROFILE_NAMES.index(name)]
        tb, ok = rocprof_summary.lookup(TRAFFIC_SUMMARY, kname, "float", items)
        if tb is None or not ok:
            measured = None
            break
        measured += tb
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
        "config": {"workload": "c3 sensor-pruned gradient evaluation: 256x256x128 cubic cells padded "
                               "512x512x256, design z<124, 64x64 sensor plane at z=127, "
                               "J=mean(Hz-0.2)^2+0.01 mean|grad_xy Hz|^2; x R2C, y FFT fused with a direct z sum "
                               "against the x-y transformed tensor (one target / source layer), inverse y, "
                               "inverse x (five kernels per evaluation)",
                   "form": "sensor-pruned (FFTs along x and y, direct sum along z)",
                   "global_batch": 1, "parallelism": "single GPU"},
        "repeats": args.repeats,
        "loops_ms_per_step": r32["loops"],
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
        # the whole evaluation on its own (sensor-pruned) byte model: the sum
        # of the five kernels' algorithmic bytes per evaluation / the step time
        "evaluation_roofline": {"bound": "hbm", "bytes_per_eval": pass_bytes,
                                "achieved": pass_bytes * evals / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": pass_bytes * evals / 1e9 / HBM_PEAK_GBS,
                                "traffic_per_eval": measured,
                                "note": "algorithmic bytes of the sensor-pruned passes; traffic = the counters "
                                        "(copy-calibrated FETCH_SIZE + WRITE_SIZE) of the same five kernels, "
                                        "null when the sources changed since they were taken"},
        # mean launch time per kernel: a burst of back-to-back launches of its
        # pass between two HIP events on its stream, median of the bursts
        "per_kernel_us": {f"{name}:{r32['kernels'][tof.PROFILE_NAMES.index(name)][0]}": round(avg * 1e3, 2)
                          for (name, avg, _, _, _) in slots},
        "per_kernel_timing": (f"burst of {args.burst_launches} launches, median of {args.bursts}"
                              if args.burst_launches > 0 else "an event per launch"),
        # every kernel's algorithmic bytes per launch / its mean launch time, of the HBM peak
        "per_kernel_frac": {f"{name}:{r32['kernels'][tof.PROFILE_NAMES.index(name)][0]}":
                            round(by / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 3) for (name, avg, _, by, _) in slots},
        "per_kernel_sum_us": round(sum(s[1] for s in slots) * 1e3, 2),
        # the same launches inside the evaluation, each with its own completion
        # event (the events lengthen every launch by a few microseconds)
        "per_kernel_us_event_per_launch": {f"{name}:{r32['kernels'][tof.PROFILE_NAMES.index(name)][0]}":
                                           round(ev * 1e3, 2) for (name, _, _, _, ev) in slots},
        "paths_f32_evals_per_s": dict({"fused": evals}, **r32["paths"]),
        "roofline": {"bound": "hbm", "kernel": f"{dom_kernel} ({dom[0]}, {dom_items} work items)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_note": traffic_note,
                     "bytes_per_launch": dom[3], "avg_launch_us": dom[1] * 1e3},
    }
    if not args.no_stream_reference:
        out["stream_reference_GBps"] = stream_reference(torch)
        print(f"[bench] streaming reference (GB/s): {out['stream_reference_GBps']}", file=sys.stderr, flush=True)
    if not args.no_full_field:
        out["full_field_pipeline"] = full_field_measurement(torch, tof, w, max(10, args.steps // 2), args.repeats,
                                                            args.burst_launches, args.bursts)
    if not args.no_batch:
        out["c5_batch"] = batch_measurement(torch, wl, args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
