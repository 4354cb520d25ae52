"""GPU tests of the differentiation form (autograd over the field and its
hand-written adjoint) and of the precision form (the projected-gradient loop
in FP32 with its error against FP64 and the oracle along the iterates)."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1707_09898_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sampled_reference(w, cells, rho=None, table=None):
    """Oracle J and the gradient at the given cells, for density rho."""
    table = oracle.table_for(w) if table is None else table
    H = oracle.forward_field(w, rho, table=table)
    J, g = oracle.objective(w, H)
    ob = oracle.objective_box(w)
    jm = oracle.objective_mask(w)
    out = []
    for (z, y, x) in cells:
        A = oracle.field(w.n, w.h, g, ob, (x, x + 1, y, y + 1, z, z + 1), jm, oracle.m0_mask(w), table)
        out.append(oracle.gradient_from_adjoint(w, A, rho)[z, y, x])
    return J, np.array(out)


def random_design_cells(w, count, seed):
    rng = np.random.default_rng(seed)
    x0, x1, y0, y1, z0, z1 = w.design
    cells = set()
    while len(cells) < count:
        cells.add((int(rng.integers(z0, z1)), int(rng.integers(y0, y1)), int(rng.integers(x0, x1))))
    return sorted(cells)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_c4_autograd_matches_finite_differences_and_oracle(torch, dtype, tol):
    """128 x 128 x 64 grid, spatially varying unit M0, J = mean over a
    32 x 32 x 4 box of |H - H*|^2 written in torch on the differentiable field:
    the backward (hand-written adjoint) against central differences (FP64,
    h = 1e-6) at 64 random design cells, against the fused
    objective_and_grad, and against the oracle."""
    from paper_1707_09898_amd import tof
    from paper_1707_09898_amd.autograd import stray_field

    w = wl.config4()
    say("c4 autograd", dtype)
    e = tof.engine_for(w, dtype)
    tdt = e.dtype
    x0, x1, y0, y1, z0, z1 = w.sensor
    S = (x1 - x0) * (y1 - y0) * (z1 - z0)
    Ht = torch.as_tensor(w.h_target, dtype=tdt, device="cuda")

    def J_of(r):
        H = stray_field(r, e)
        d = H[:, z0:z1, y0:y1, x0:x1] - Ht
        return (d * d).sum() / S

    rho = torch.as_tensor(w.rho, dtype=tdt, device="cuda").requires_grad_(True)
    J = J_of(rho)
    J.backward()
    g = rho.grad.detach().cpu().numpy().astype(np.float64)
    cells = random_design_cells(w, 64, 4)
    # the fused path computes the same gradient
    Jf, gf = e.objective_and_grad(rho.detach().contiguous())
    torch.cuda.synchronize()
    gf = gf.cpu().numpy().astype(np.float64)
    assert abs(Jf.item() - J.item()) <= tol * abs(J.item())
    assert np.abs(gf - g).max() <= tol * np.abs(g).max()
    # oracle at the sampled cells
    Jr, gr = sampled_reference(w, cells)
    assert abs(J.item() - Jr) <= tol * abs(Jr)
    got = np.array([g[c] for c in cells])
    assert np.abs(got - gr).max() <= tol * np.abs(gr).max()
    if dtype == "f64":
        h = 1e-6
        fd = []
        with torch.no_grad():
            for c in cells:
                vals = []
                for s in (+1.0, -1.0):
                    r = rho.detach().clone()
                    r[c] += s * h
                    vals.append(J_of(r).item())
                fd.append((vals[0] - vals[1]) / (2 * h))
        fd = np.array(fd)
        scale = np.abs(gr).max()
        err = np.abs(got - fd).max()
        say(f"  FD max err {err:.3e} (grad scale {scale:.3e})")
        assert err <= 1e-6 * scale + 1e-12


def test_c3_precision_loop(torch):
    """200 projected-gradient iterations in FP32 on 256 x 256 x 128 (rho
    clamped to [0, 1]); every 20 iterations the FP32 gradient is compared with
    the plain FP64 GPU path on the same iterate, and at iterations 0, 100 and
    200 both are compared with the oracle's J and whole gradient on that
    iterate.

    Bar, at every compared iterate and relative to that iterate's own
    gradient (max |g - g_ref| / max |g_ref|): FP64 within 1e-10 of the
    oracle; FP32 within 1e-5 of the FP64 path and of the oracle, on J and on
    the gradient.  The error against the starting gradient scale is reported
    as well."""
    from paper_1707_09898_amd import tof

    w = wl.config3()
    e32 = tof.engine_for(w, "f32")
    e64 = tof.engine_for(w, "f64")
    rho = torch.as_tensor(w.rho, dtype=torch.float32, device="cuda")
    g32 = torch.empty_like(rho)
    J32 = torch.empty(1, dtype=torch.float64, device="cuda")
    table = oracle.table_for(w)
    report = []
    Js = []
    gscale0 = None
    for k in range(201):
        e32.objective_and_grad(rho, g32, J32)
        if k % 20 == 0:
            r64 = rho.double()
            J64, g64 = e64.objective_and_grad(r64)
            torch.cuda.synchronize()
            a32 = g32.cpu().numpy().astype(np.float64)
            a64 = g64.cpu().numpy()
            if gscale0 is None:
                gscale0 = float(np.abs(a64).max())
            e_abs = float(np.abs(a32 - a64).max())
            e_g = e_abs / float(np.abs(a64).max())
            e_j = abs(J32.item() - J64.item()) / abs(J64.item())
            row = {"iter": k, "J32": J32.item(), "J64": J64.item(), "relJ_32_vs_64": e_j, "relgrad_32_vs_64": e_g,
                   "grad_err_vs_start_scale": e_abs / gscale0}
            if k in (0, 100, 200):
                rho_np = r64.cpu().numpy()
                t0 = time.perf_counter()
                Jr, gr, _ = oracle.objective_and_grad(w, rho_np, table)
                gs = float(np.abs(gr).max())
                row.update({"relJ_32_vs_oracle": abs(J32.item() - Jr) / abs(Jr),
                            "relJ_64_vs_oracle": abs(J64.item() - Jr) / abs(Jr),
                            "relgrad_32_vs_oracle": float(np.abs(a32 - gr).max()) / gs,
                            "relgrad_64_vs_oracle": float(np.abs(a64 - gr).max()) / gs,
                            "oracle_s": time.perf_counter() - t0})
                assert row["relJ_64_vs_oracle"] <= 1e-10 and row["relgrad_64_vs_oracle"] <= 1e-10, row
                assert row["relJ_32_vs_oracle"] <= 1e-5 and row["relgrad_32_vs_oracle"] <= 1e-5, row
            say("  " + " ".join(f"{kk}={v:.3e}" if isinstance(v, float) else f"{kk}={v}" for kk, v in row.items()))
            report.append(row)
            assert e_j <= 1e-5 and e_g <= 1e-5, row
        Js.append(J32.item())
        e32.project_step(rho, g32, 0.05)
    # the loop makes progress and keeps rho in [0, 1]
    assert Js[-1] < Js[0]
    assert float(rho.min()) >= 0.0 and float(rho.max()) <= 1.0
