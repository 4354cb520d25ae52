"""Schedule autotuner: padded lengths, pass structure and tile knobs.

Any padded length L >= 2n - 1 gives the same (exact) convolution, so the
length per axis is a free schedule choice: the default is the smallest even
7-smooth L >= 2n (mixed-radix LDS transforms for non-powers of two), while a
power of two in [32, 512] selects the register-resident transforms and, for
the y axis, the fused y / z-sum kernels, at the price of a longer line.  The
pass structure is free too (the same convolution up to rounding order):
the fused y / z-sum kernels, the direct z sum in a pass of its own, or FFTs
along z.  tune() times gradient evaluations per candidate length triple,
tune_schedule() per (triple, pass structure) pair, on the GPU, and keeps the
fastest; results are cached per (grid, cell, objective) key.  tune_batch()
picks the tile knobs of the batched form per padded length (x-pass tile per
Lx, row groups of the fused gather and scatter per Ly) by timing whole
batched evaluations.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

MAX_L = 1024


def smooth7(L: int) -> bool:
    if L < 1:
        return False
    for f in (2, 3, 5, 7):
        while L % f == 0:
            L //= f
    return L == 1


def default_length(n: int) -> int:
    """The library's rule: the smallest even 7-smooth L >= 2n."""
    L = 2 * n
    while not smooth7(L):
        L += 2
    return L


def candidate_lengths(n: int) -> List[int]:
    """Padded lengths worth timing for an axis of n cells: the default rule,
    and the smallest power of two >= 2n - 1 when it differs (and fits)."""
    out = [default_length(n)]
    p2 = 1
    while p2 < 2 * n - 1:
        p2 *= 2
    p2 = max(p2, 2)
    if p2 != out[0] and p2 <= MAX_L:
        out.append(p2)
    return out


def candidate_triples(n: Sequence[int]) -> List[Tuple[int, int, int]]:
    """The default triple, powers of two on every axis, and a power of two on
    y only (the axis that decides the fused y / z-sum path); duplicates dropped."""
    d = [default_length(v) for v in n]
    p = [candidate_lengths(v)[-1] for v in n]
    out = []
    for t in (tuple(d), tuple(p), (d[0], p[1], d[2])):
        if t not in out:
            out.append(t)
    return out


# pass structures: (TOF_OPT_ZSUM, TOF_OPT_FUSE_YZ, TOF_OPT_FUSE_OBJECTIVE)
PASSES = {"fused": (1, 1, 1), "zsum": (1, 0, 1), "zfft": (0, 0, 1)}

_CACHE: Dict[tuple, Tuple[int, int, int]] = {}
_SCHED: Dict[tuple, Tuple[Tuple[int, int, int], str]] = {}


def key_of(w, dtype: str) -> tuple:
    return (tuple(w.n), tuple(round(v, 12) for v in w.h), tuple(w.design), tuple(w.sensor), w.j_kind, dtype)


def tune(w, dtype: str = "f32", evals: int = 3, candidates=None) -> Tuple[Tuple[int, int, int], Dict]:
    """Time `evals` gradient evaluations for every candidate length triple of
    workload w; returns (best triple, {triple: ms per evaluation})."""
    import torch
    from . import tof
    key = key_of(w, dtype)
    cands = candidate_triples(w.n) if candidates is None else list(candidates)
    times = {}
    for L in cands:
        e = tof.engine_for(w, dtype, L=L)
        rho = torch.as_tensor(w.rho, dtype=e.dtype, device="cuda")
        grad = torch.empty_like(rho)
        J = torch.empty(1, dtype=torch.float64, device="cuda")
        e.objective_and_grad(rho, grad, J)   # warm-up
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(evals):
            e.objective_and_grad(rho, grad, J)
        t1.record()
        torch.cuda.synchronize()
        times[tuple(L)] = t0.elapsed_time(t1) / evals
        e.close()
    best = min(times, key=times.get)
    _CACHE[key] = best
    return best, times


def cached(w, dtype: str = "f32"):
    """The tuned lengths of a workload if tune() has seen it, else None."""
    return _CACHE.get(key_of(w, dtype))


def apply_passes(e, name: str):
    """Set the pass structure `name` (a key of PASSES) on engine e."""
    from . import tof
    zsum, fuse, fobj = PASSES[name]
    e.set_option(tof.OPT_ZSUM, zsum)
    e.set_option(tof.OPT_FUSE_YZ, fuse)
    e.set_option(tof.OPT_FUSE_OBJECTIVE, fobj)


def tune_schedule(w, dtype: str = "f32", evals: int = 3, candidates=None, passes=None):
    """Time `evals` gradient evaluations for every (length triple, pass
    structure) pair of workload w; returns ((triple, pass name),
    {(triple, pass name): ms per evaluation})."""
    import torch
    from . import tof
    key = key_of(w, dtype)
    cands = candidate_triples(w.n) if candidates is None else list(candidates)
    names = list(PASSES) if passes is None else list(passes)
    times = {}
    for L in cands:
        e = tof.engine_for(w, dtype, L=L)
        rho = torch.as_tensor(w.rho, dtype=e.dtype, device="cuda")
        grad = torch.empty_like(rho)
        J = torch.empty(1, dtype=torch.float64, device="cuda")
        for name in names:
            apply_passes(e, name)
            e.objective_and_grad(rho, grad, J)   # warm-up
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(evals):
                e.objective_and_grad(rho, grad, J)
            t1.record()
            torch.cuda.synchronize()
            times[(tuple(L), name)] = t0.elapsed_time(t1) / evals
        e.close()
    best = min(times, key=times.get)
    _SCHED[key] = best
    _CACHE[key] = best[0]
    return best, times


# tile knobs of the batched form, the candidates tried per padded length
BATCH_KNOBS = {
    "x_tile": (lambda L: [1, 2]),                       # full tile, one row pair a block
    "gather_groups": (lambda L: [1, 2, 3, 4, 6, 8]),
    "scatter_groups": (lambda L: [1, 2, 4, 8]),
}


def _knob_option(name):
    from . import tof
    return {"x_tile": tof.OPT_X_TILE, "gather_groups": tof.OPT_GATHER_GROUPS,
            "scatter_groups": tof.OPT_SCATTER_GROUPS}[name]


def _knob_axis(name):
    return 0 if name == "x_tile" else 1   # the x tile follows Lx; the fused y / z sums follow Ly


def apply_batch_knobs(b, table):
    """Set table[name][L] on every engine of batch b whose padded length
    along the knob's axis is L, then re-record the batch."""
    for e in b.engines:
        L = e.padded_lengths()
        for name, per_len in table.items():
            v = per_len.get(L[_knob_axis(name)])
            if v is not None:
                e.set_option(_knob_option(name), int(v))
    b.rebatch()


def tune_batch(b, evals: int = 5, rounds: int = 1):
    """Coordinate search over the tile knobs of a batched DesignBatch: for
    every knob and every padded length present along its axis, each
    candidate value is timed on the whole batch (eager launches, median of 3
    loops) and the fastest kept.  Returns (table {knob: {L: value}}, best ms,
    {(knob, L, value): ms})."""
    lens = {name: sorted({e.padded_lengths()[_knob_axis(name)] for e in b.engines}) for name in BATCH_KNOBS}
    table = {name: {L: BATCH_KNOBS[name](L)[0] for L in lens[name]} for name in BATCH_KNOBS}
    apply_batch_knobs(b, table)
    best = b.time_eager(evals)
    trials = {}
    for _ in range(rounds):
        for name in BATCH_KNOBS:
            for L in lens[name]:
                keep = table[name][L]
                for v in BATCH_KNOBS[name](L):
                    if v == keep:
                        continue
                    table[name][L] = v
                    apply_batch_knobs(b, table)
                    ms = b.time_eager(evals)
                    trials[(name, L, v)] = ms
                    if ms < best:
                        best, keep = ms, v
                table[name][L] = keep
                apply_batch_knobs(b, table)
    return table, best, trials
