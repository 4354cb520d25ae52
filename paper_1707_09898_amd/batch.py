"""Batching form: many independent designs, each with its own context, run
as one HIP graph.

Every design keeps its density, gradient and J resident on the device.  The
gradient evaluations are recorded once into a graph (torch.cuda.CUDAGraph
over the library's own launches): the designs are spread over several
streams forked from the capture stream (balanced by padded volume), so
independent designs overlap on the GPU, and one replay evaluates the whole
batch.  Each context owns its
workspaces, so concurrent designs share nothing.
"""
from __future__ import annotations

from typing import List, Optional, Sequence


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
                 streams: int = 4, passes: Optional[Sequence[str]] = None):
        import torch
        from . import autotune, tof
        self.torch = torch
        self.workloads = list(workloads)
        self.dtype = dtype
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
        """Fork the side streams from `root`, enqueue every design, join back."""
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
        for e in self.engines:
            e.close()
        self.engines = []
