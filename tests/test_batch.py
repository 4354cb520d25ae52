"""The batching form: independent designs of uneven size run as one HIP graph
(graph replays against eager launches and against the oracle), and the
padded-length autotuner (its candidate rule on the CPU; tuned lengths give
the same result on the GPU)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1707_09898_amd import autotune
from paper_1707_09898_amd import workloads as wl


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def smallest_designs(count):
    ws = wl.config5()
    order = sorted(range(len(ws)), key=lambda i: int(np.prod(ws[i].n)))
    return [ws[i] for i in order[:count]]


# ---------------------------------------------------------------- CPU
def brute_smooth7(L):
    return L >= 1 and all(p in (2, 3, 5, 7) for p in prime_factors(L))


def prime_factors(L):
    out, d = [], 2
    while d * d <= L:
        while L % d == 0:
            out.append(d)
            L //= d
        d += 1
    if L > 1:
        out.append(L)
    return out


@pytest.mark.parametrize("n", [1, 2, 16, 33, 37, 64, 97, 101, 160, 257, 512])
def test_candidate_lengths_are_valid(n):
    cands = autotune.candidate_lengths(n)
    assert cands[0] == min(L for L in range(2 * n, 4 * n + 8, 2) if brute_smooth7(L))
    for L in cands:
        assert L % 2 == 0 and L >= 2 * n - 1 and L <= autotune.MAX_L and brute_smooth7(L)
    if len(cands) > 1:
        assert cands[1] & (cands[1] - 1) == 0


def test_balance_assigns_every_design_once_and_evens_the_streams():
    from paper_1707_09898_amd.batch import balance
    rng = np.random.default_rng(7)
    cost = [float(v) for v in rng.integers(1, 1000, size=64)]
    for ns in (1, 2, 4, 8):
        out = balance(cost, ns)
        assert len(out) == ns
        assert sorted(i for s in out for i in s) == list(range(len(cost)))
        loads = [sum(cost[i] for i in s) for s in out]
        # largest-first greedy: no stream exceeds the mean by more than the largest cost
        assert max(loads) <= sum(cost) / ns + max(cost)
        for s in out:   # each stream runs its designs largest first
            assert all(cost[a] >= cost[b] for a, b in zip(s, s[1:]))


def test_candidate_triples_start_with_the_default():
    t = autotune.candidate_triples((37, 64, 33))
    assert t[0] == (80, 128, 70) and (128, 128, 128) in t and len(set(t)) == len(t)


# ---------------------------------------------------------------- GPU
@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["batched", "streams"])
def test_graph_replays_match_eager_launches(torch, mode):
    """Six designs of the 64-design batch (batched launches, or each design's
    own launches on three streams): every replay of the captured graph
    reproduces the eager results bit for bit, with other device work and
    synchronizations between the replays."""
    from paper_1707_09898_amd.batch import DesignBatch
    ws = smallest_designs(6)
    say("batch graph", mode, [w.n for w in ws])
    b = DesignBatch(ws, "f32", streams=3, mode=mode)
    b.run_eager()
    ref = b.results()
    b.capture()
    for k in range(3):
        for g in b.grad:
            g.fill_(float("nan"))
        for J in b.J:
            J.fill_(float("nan"))
        torch.cuda.synchronize()
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()   # the program's own eager work between replays
        b.replay()
        got = b.results()
        for (J0, g0), (J1, g1) in zip(ref, got):
            assert J0 == J1 and np.array_equal(g0, g1), k
    b.close()


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_batch_matches_oracle(torch, dtype, tol):
    """The two smallest designs of the batch, evaluated by a graph replay of
    the batched launches, against the oracle's J and full gradient."""
    from paper_1707_09898_amd.batch import DesignBatch
    ws = smallest_designs(2)
    b = DesignBatch(ws, dtype, streams=2)
    b.capture()
    b.replay()
    got = b.results()
    b.close()
    for w, (J, g) in zip(ws, got):
        say("batch oracle", dtype, w.n, w.p)
        Jr, gr, _ = oracle.objective_and_grad(w)
        assert abs(J - Jr) <= tol * abs(Jr)
        assert np.abs(g.astype(np.float64) - gr).max() <= tol * np.abs(gr).max()


@pytest.mark.gpu
def test_tuned_lengths_give_the_same_result(torch):
    """Every candidate length triple of a design gives the same J and
    gradient (FP64, to 1e-12), and the tuner returns one of them."""
    from paper_1707_09898_amd import tof
    w = smallest_designs(1)[0]
    best, times = autotune.tune(w, "f64", evals=2)
    say("tuned", w.n, best, times)
    assert best in times and len(times) == len(autotune.candidate_triples(w.n))
    res = []
    for L in times:
        e = tof.engine_for(w, "f64", L=L)
        assert e.padded_lengths() == tuple(L)
        J, g = e.objective_and_grad(torch.as_tensor(w.rho, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        res.append((J.item(), g.cpu().numpy()))
        e.close()
    J0, g0 = res[0]
    for J, g in res[1:]:
        assert abs(J - J0) <= 1e-12 * abs(J0)
        assert np.abs(g - g0).max() <= 1e-12 * np.abs(g0).max()


@pytest.mark.gpu
def test_tuned_schedules_give_the_same_result(torch):
    """The schedule tuner times every (length triple, pass structure) pair,
    returns one of them, and a batch built from tuned schedules matches the
    same designs evaluated one by one with the library's defaults."""
    from paper_1707_09898_amd import tof
    from paper_1707_09898_amd.batch import DesignBatch
    ws = smallest_designs(3)
    sched = []
    for w in ws:
        best, times = autotune.tune_schedule(w, "f64", evals=1)
        say("schedule", w.n, best)
        assert best in times
        assert len(times) == len(autotune.candidate_triples(w.n)) * len(autotune.PASSES)
        sched.append(best)
    b = DesignBatch(ws, "f64", [L for L, _ in sched], streams=2, passes=[p for _, p in sched], mode="streams")
    b.run_eager()
    got = b.results()
    b.close()
    for w, (J, g) in zip(ws, got):
        e = tof.engine_for(w, "f64")
        J0, g0 = e.objective_and_grad(torch.as_tensor(w.rho, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        g0 = g0.cpu().numpy()
        e.close()
        assert abs(J - J0.item()) <= 1e-12 * abs(J0.item())
        assert np.abs(g - g0).max() <= 1e-12 * np.abs(g0).max()


def c5_reference(cache):
    """Oracle J and full gradient of all 64 designs of the batch (FP64)."""
    if "c5" not in cache:
        import time
        t0 = time.perf_counter()
        cache["c5"] = [oracle.objective_and_grad(w)[:2] for w in wl.config5()]
        say(f"oracle: 64 designs in {time.perf_counter() - t0:.1f} s")
    return cache["c5"]


@pytest.mark.gpu
def test_whole_batch_with_tuned_schedules_matches_oracle(torch, oracle_cache):
    """All 64 designs, with the schedules the tuner picks (as the benchmark
    runs them), evaluated by one graph replay in FP32: J and the whole
    gradient of every design against the oracle at 1e-5."""
    from paper_1707_09898_amd.batch import DesignBatch
    ws = wl.config5()
    sched = [autotune.tune_schedule(w, "f32", evals=2)[0] for w in ws]
    b = DesignBatch(ws, "f32", [L for L, _ in sched], streams=4, passes=[p for _, p in sched], mode="streams")
    b.capture()
    b.replay()
    got = b.results()
    b.close()
    ref = c5_reference(oracle_cache)
    worst = 0.0
    for i, (w, (J, g), (Jr, gr)) in enumerate(zip(ws, got, ref)):
        eJ = abs(J - Jr) / abs(Jr)
        eg = float(np.abs(g.astype(np.float64) - gr).max() / np.abs(gr).max())
        worst = max(worst, eJ, eg)
        assert eJ <= 1e-5 and eg <= 1e-5, (i, w.name, sched[i], eJ, eg)
    say(f"batch: worst relative error over 64 designs {worst:.2e}")


@pytest.mark.gpu
def test_batched_form_whole_batch_matches_oracle_and_single_launches(torch, oracle_cache):
    """All 64 designs in the batched form (one launch per pass and kernel
    instantiation, over device tables of the designs' arguments), one graph
    replay in FP32: J and the whole gradient of every design against the
    oracle at 1e-5, and against the same design evaluated alone with the same
    padded lengths (the same kernels: equal to rounding)."""
    from paper_1707_09898_amd import tof
    from paper_1707_09898_amd.batch import DesignBatch, batch_lengths
    ws = wl.config5()
    b = DesignBatch(ws, "f32")
    n_launch = b.launches()
    say(f"batched form: {n_launch} launches for {len(ws)} designs")
    assert n_launch <= 5 * 12
    b.capture()
    b.replay()
    got = b.results()
    b.close()
    ref = c5_reference(oracle_cache)
    worst = 0.0
    for i, (w, (J, g), (Jr, gr)) in enumerate(zip(ws, got, ref)):
        eJ = abs(J - Jr) / abs(Jr)
        eg = float(np.abs(g.astype(np.float64) - gr).max() / np.abs(gr).max())
        worst = max(worst, eJ, eg)
        assert eJ <= 1e-5 and eg <= 1e-5, (i, w.name, eJ, eg)
    say(f"batched form: worst relative error over 64 designs {worst:.2e}")
    for i in (0, 17, 63):
        w = ws[i]
        e = tof.engine_for(w, "f32", L=batch_lengths(w))
        J1, g1 = e.objective_and_grad(torch.as_tensor(w.rho, dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        g1 = g1.cpu().numpy()
        e.close()
        J, g = got[i]
        assert abs(J - J1.item()) <= 1e-6 * abs(J1.item())
        assert np.abs(g - g1).max() <= 1e-6 * np.abs(g1).max()


@pytest.mark.gpu
def test_tuned_batched_form_matches_oracle(torch, oracle_cache):
    """The tile knobs the batch tuner picks per padded length (x tile, gather
    and scatter row groups) change only the work split (and the order of the
    gather's partial sums): all 64 designs still match the oracle at 1e-5,
    graph replays included."""
    from paper_1707_09898_amd import autotune
    from paper_1707_09898_amd.batch import DesignBatch
    ws = wl.config5()
    b = DesignBatch(ws, "f32")
    table, best, trials = autotune.tune_batch(b, evals=3)
    say(f"batch tuner: {best:.3f} ms, {len(trials)} trials, {table}")
    assert set(table) == set(autotune.BATCH_KNOBS)
    b.capture()
    b.replay()
    b.replay()
    got = b.results()
    b.close()
    ref = c5_reference(oracle_cache)
    for i, (w, (J, g), (Jr, gr)) in enumerate(zip(ws, got, ref)):
        assert abs(J - Jr) <= 1e-5 * abs(Jr), (i, w.name)
        assert np.abs(g.astype(np.float64) - gr).max() <= 1e-5 * np.abs(gr).max(), (i, w.name)
