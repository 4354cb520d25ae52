"""The allocation-free projected step (tof_project_step_static, for callers
that cannot allocate) against the context's tof_project_step: the same
update, bit for bit, on two calls in a row, the second on a smaller grid
(the static scratch keeps the first call's partial maxima, which the second
must not read), with and without a design mask, in FP32 and FP64."""
import sys

import numpy as np
import pytest

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


def step_both(torch, w, dtype, alpha):
    """(result of the context's step, result of the static step) on the
    workload's density and a seeded gradient."""
    from paper_1707_09898_amd import tof
    tdt = torch.float32 if dtype == "f32" else torch.float64
    rng = np.random.default_rng(w.n[0] * 1000 + w.n[1])
    gh = rng.normal(size=w.rho.shape)
    rho_a = torch.as_tensor(w.rho, dtype=tdt).cuda()
    rho_b = rho_a.clone()
    grad = torch.as_tensor(gh, dtype=tdt).cuda()
    mask = None if w.mask is None else torch.as_tensor(w.mask, dtype=torch.uint8).cuda()
    e = tof.Engine(w.n, w.h, dtype)
    e.set_design(w.design, p=w.p, mask=mask)
    e.project_step(rho_a, grad, alpha)
    tof.project_step_static(rho_b, grad, alpha, design=w.design, mask=mask)
    torch.cuda.synchronize()
    e.close()
    return rho_a.cpu().numpy(), rho_b.cpu().numpy()


@pytest.mark.parametrize("with_mask", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_static_step_equals_context_step_twice_second_smaller(torch, dtype, with_mask):
    big = wl.small_random(71, n=(96, 80, 40), design=(3, 90, 0, 80, 0, 33))
    small = wl.small_random(72, n=(9, 7, 6), design=(1, 8, 1, 7, 0, 5))
    for w in (big, small):
        if with_mask:
            w.mask = wl.random_mask(w.n[0], w.n, 0.6)
        say("static step", dtype, with_mask, w.n)
        a, b = step_both(torch, w, dtype, 0.07)
        assert np.array_equal(a, b), float(np.abs(a - b).max())
        assert not np.array_equal(a, w.rho.astype(a.dtype))   # the step moved something


def test_static_step_rejects_bad_arguments(torch):
    from paper_1707_09898_amd import tof
    rho = torch.zeros((4, 4, 4), dtype=torch.float32, device="cuda")
    g = torch.ones_like(rho)
    with pytest.raises(tof.TofError):
        tof.project_step_static(rho, g, -1.0)
    with pytest.raises(tof.TofError):
        tof.project_step_static(rho, g, 0.1, design=(0, 5, 0, 4, 0, 4))
    import ctypes
    L = tof.lib()
    big = tof.make_grid((600, 4, 4), (1, 1, 1), "f32")
    st = L.tof_project_step_static(ctypes.byref(big), None, None, ctypes.c_void_p(rho.data_ptr()),
                                   ctypes.c_void_p(g.data_ptr()), 0.1, None)
    assert st == -1 and b"512" in L.tof_last_error(None)
    ok = tof.make_grid((4, 4, 4), (1, 1, 1), "f32")
    assert L.tof_project_step_static(ctypes.byref(ok), None, None, None, ctypes.c_void_p(g.data_ptr()), 0.1,
                                     None) == -1
