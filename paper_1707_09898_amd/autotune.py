"""Padded-length autotuner.

Any padded length L >= 2n - 1 gives the same (exact) convolution, so the
length per axis is a free schedule choice: the default is the smallest even
7-smooth L >= 2n (mixed-radix LDS transforms for non-powers of two), while a
power of two in [32, 512] selects the register-resident transforms and, for
the y axis, the fused y / z-sum kernels, at the price of a longer line.  The
tuner times one gradient evaluation per candidate triple on the GPU and keeps
the fastest; results are cached per (grid, cell, objective) key.
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


_CACHE: Dict[tuple, Tuple[int, int, int]] = {}


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
