"""Batching form: many independent designs, each with its own context,
evaluated together.

Every design keeps its density, gradient and J resident on the device.  Two
modes:

* ``batched`` (default): the library's batched form (tof_batch): one launch
  per pass and kernel instantiation for all designs, each launch over a
  device table of the designs' arguments, so the whole batch is a handful
  of launches (designs with the same padded lengths share them).  It needs
  the fused passes, hence power-of-two padded lengths along x and y
  (``batch_lengths``).
* ``streams``: every design's own five launches, spread over several streams
  forked from the capture stream (balanced by padded volume), so
  independent designs overlap on the GPU.

Either way one evaluation of the batch can be recorded into a graph
(torch.cuda.CUDAGraph over the library's own launches) and replayed.  Each
context owns its workspaces, so concurrent designs share nothing.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple


def pow2_at_least(v: int, lo: int = 32) -> int:
    p = lo
    while p < v:
        p *= 2
    return p


def batch_lengths(w, floor: int = 32) -> Tuple[int, int, int]:
    """Padded lengths for the batched form: the smallest powers of two
    >= 2n - 1 along x and y, and at least `floor` (>= 32; the fused kernels'
    register transforms), the library's rule along z (the fused passes sum
    along z directly and never transform along it).  A higher floor puts
    small designs into the launches of larger ones (fewer launches, more
    bytes)."""
    from .autotune import default_length
    nx, ny, nz = w.n
    lo = max(32, int(floor))
    return (pow2_at_least(2 * nx - 1, lo), pow2_at_least(2 * ny - 1, lo), default_length(nz))


def balance(cost: Sequence[float], nstreams: int) -> List[List[int]]:
    """Indices per stream: largest cost first, each to the stream with the
    least cost so far, so that the streams end at about the same time."""
    order = sorted(range(len(cost)), key=lambda i: -cost[i])
    load = [0.0] * nstreams
    out: List[List[int]] = [[] for _ in range(nstreams)]
    for i in order:
        k = min(range(nstreams), key=lambda s: load[s])
        out[k].append(i)
        load[k] += cost[i]
    return out


class DesignBatch:
    def __init__(self, workloads: Sequence, dtype: str = "f32", lengths: Optional[Sequence] = None,
                 streams: int = 4, passes: Optional[Sequence[str]] = None, mode: str = "batched"):
        import torch
        from . import autotune, tof
        if mode not in ("batched", "streams"):
            raise ValueError("mode is 'batched' or 'streams'")
        self.torch = torch
        self.mode = mode
        self.workloads = list(workloads)
        self.dtype = dtype
        if mode == "batched":
            if lengths is None:
                lengths = [batch_lengths(w) for w in self.workloads]
            if passes is not None and any(p != "fused" for p in passes):
                raise ValueError("the batched mode runs the fused passes only")
        self.engines = []
        self.rho, self.grad, self.J = [], [], []
        for i, w in enumerate(self.workloads):
            L = None if lengths is None else lengths[i]
            e = tof.engine_for(w, dtype, L=L)
            if passes is not None:
                autotune.apply_passes(e, passes[i])
            self.engines.append(e)
            r = torch.as_tensor(w.rho, dtype=e.dtype, device="cuda")
            self.rho.append(r)
            self.grad.append(torch.empty_like(r))
            self.J.append(torch.empty(1, dtype=torch.float64, device="cuda"))
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        self.assignment = self._balance(len(self.streams))
        self.graph = None
        self.batch = tof.Batch(self.engines, self.rho, self.J, self.grad) if mode == "batched" else None

    def rebatch(self):
        """Record the batched launches again (after a change of the engines'
        options); any captured graph is dropped."""
        from . import tof
        self.graph = None
        if self.batch is not None:
            self.batch.close()
        self.batch = tof.Batch(self.engines, self.rho, self.J, self.grad)

    def time_eager(self, evals: int = 5, repeats: int = 3) -> float:
        """ms per batch evaluation launched eagerly (median of `repeats` loops)."""
        torch = self.torch
        self.run_eager()
        out = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(evals):
                self.run_eager()
            t1.record()
            torch.cuda.synchronize()
            out.append(t0.elapsed_time(t1) / evals)
        return sorted(out)[len(out) // 2]

    def launches(self) -> int:
        """Kernel launches of one evaluation of the batch."""
        return self.batch.launches() if self.batch is not None else 5 * len(self.engines)

    def _balance(self, nstreams: int) -> List[List[int]]:
        """Designs per stream, balanced by padded volume (see balance)."""
        cost = []
        for e in self.engines:
            Lx, Ly, Lz = e.padded_lengths()
            cost.append(Lx * Ly * Lz)
        return balance(cost, nstreams)

    def __len__(self):
        return len(self.engines)

    def _enqueue(self, root):
        """Enqueue one evaluation of every design on `root` (batched), or fork
        the side streams from `root`, enqueue every design, join back."""
        if self.batch is not None:
            self.batch.run(stream=root)
            return
        for s in self.streams:
            s.wait_stream(root)
        for s, designs in zip(self.streams, self.assignment):
            for i in designs:
                self.engines[i].objective_and_grad(self.rho[i], self.grad[i], self.J[i], stream=s)
        for s in self.streams:
            root.wait_stream(s)

    def run_eager(self):
        """One evaluation of every design, launched directly (no graph)."""
        self._enqueue(self.torch.cuda.current_stream())

    def capture(self):
        """Record one evaluation of every design into a graph."""
        torch = self.torch
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=cap):
            self._enqueue(torch.cuda.current_stream())
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def results(self):
        """[(J, grad)] per design, on the host (synchronizes)."""
        self.torch.cuda.synchronize()
        return [(float(self.J[i].item()), self.grad[i].detach().cpu().numpy()) for i in range(len(self))]

    def algorithmic_bytes(self) -> float:
        """Sum over the designs of one evaluation's pass bytes (from one profiled eager run)."""
        total = 0.0
        for i, e in enumerate(self.engines):
            e.profile(True)
            e.objective_and_grad(self.rho[i], self.grad[i], self.J[i])
            prof = e.profile_read()
            e.profile(False)
            total += sum(by for (_, _, cnt, by) in prof if cnt > 0)
        return total

    def close(self):
        self.graph = None
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        for e in self.engines:
            e.close()
        self.engines = []
