"""The paper's benchmark problem (maximize Hz above a cube, rho = 1 start,
L-BFGS-B on the host, GPU gradients): geometry on the CPU; on the GPU, the
starting gradient against the oracle and a short optimization run."""
import numpy as np
import pytest

import oracle
from paper_1707_09898_amd import experiments as ex
from paper_1707_09898_amd import workloads as wl


def test_benchmark_geometry():
    w = ex.benchmark_workload(1)
    assert w.n == (39, 39, 41) and w.cells == 62361          # the paper's FD mesh size
    assert w.design == (0, 39, 0, 39, 0, 39)
    assert w.sensor == (13, 26, 13, 26, 39, 41)               # centred above the cube
    assert w.j_kind == wl.J_NEG_HALF_HZ2 and w.p == 3 and np.all(w.rho == 1.0)
    w2 = ex.benchmark_workload(2)
    assert w2.n == (78, 78, 82) and abs(w2.h[0] - 1 / 78) < 1e-15


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.mark.gpu
def test_benchmark_start_gradient_matches_oracle(torch):
    """At rho = 1 on the 39 x 39 x 41 benchmark: J and dJ/drho (FP64) within
    1e-10 of the oracle; material right under the box helps (negative
    derivative), and some material elsewhere hurts (positive), which is why
    the optimization removes material."""
    from paper_1707_09898_amd import tof
    w = ex.benchmark_workload(1)
    e = tof.engine_for(w, "f64")
    J, g = e.objective_and_grad(torch.as_tensor(w.rho, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    Jr, gr, _ = oracle.objective_and_grad(w)
    assert abs(J.item() - Jr) <= 1e-10 * abs(Jr)
    assert np.abs(g - gr).max() <= 1e-10 * np.abs(gr).max()
    assert J.item() < 0
    assert g[38, 19, 19] < 0 and g.max() > 0


@pytest.mark.gpu
def test_short_benchmark_optimization(torch):
    """Ten L-BFGS-B iterations on a 13 x 13 x 15 version: J falls, rho stays in
    [0, 1], the volume fraction leaves 1."""
    c = 13
    w = wl.Workload(name="bench_small", n=(c, c, c + 2), h=(1 / c,) * 3, design=(0, c, 0, c, 0, c),
                    sensor=(4, 9, 4, 9, c, c + 2), p=3, rho=np.ones((c + 2, c, c)),
                    j_kind=wl.J_NEG_HALF_HZ2, j_target=0.0, j_lambda=0.0)
    r = ex.optimize(w, "f64", maxiter=10)
    Js = [h["J"] for h in r["history"]]
    assert r["J_best"] < Js[0] and r["iterations"] >= 5
    assert 0.0 < r["volume_fraction_final"] < 1.0
    assert sum(r["rho_histogram"]["counts"]) == c ** 3


@pytest.mark.gpu
def test_field_gradient_design_start_gradient_matches_oracle(torch):
    """The field and gradient design at rho = 1 (64 x 64 x 33, field region
    20 x 20, strip on three sides): J and dJ/drho (FP64) within 1e-10 of the
    oracle, with the weight that balances the two terms."""
    from paper_1707_09898_amd import tof
    beta = ex.balanced_beta(ex.field_gradient_workload())
    assert beta > 0
    w = ex.field_gradient_workload(beta)
    e = tof.engine_for(w, "f64")
    J, g = e.objective_and_grad(torch.as_tensor(w.rho, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    Jr, gr, _ = oracle.objective_and_grad(w)
    assert abs(J.item() - Jr) <= 1e-10 * abs(Jr)
    assert np.abs(g - gr).max() <= 1e-10 * np.abs(gr).max()
