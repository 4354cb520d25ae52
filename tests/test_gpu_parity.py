"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on seeded inputs (small and ragged sizes that span several tiles),
and on the whole gradient at the full 256 x 256 x 128 size on every pass
choice (the fused one in the launch configuration the benchmark times);
boundary behaviour (validation, the setup self-check, workspace sizing).

Tolerances (normwise, max|x - ref| / max|ref|): 1e-10 in FP64 and 1e-5 in
FP32, the accuracy targets of the gradient engine; J relative to |J|.
"""
import dataclasses
import sys
import time

import ctypes

import numpy as np
import pytest

import oracle
from paper_1707_09898_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def tof():
    from paper_1707_09898_amd import tof as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_inf(x, ref):
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


# pass choices: the fused kernels (y transforms with the direct z sum, the
# objective with the adjoint's x pass), the direct z sum in its own pass with
# the objective in its own kernel, FFTs along z
# (TOF_OPT_ZSUM, TOF_OPT_FUSE_YZ, TOF_OPT_FUSE_OBJECTIVE)
PATHS = {"fused": (1, 1, 1), "zsum": (1, 0, 0), "zfft": (0, 0, 0)}
# the gradient also with the objective fused but the y / z passes not (the
# adjoint then ends without the fused scatter, and a kernel of its own forms
# J from the objective's block sums)
GRAD_PATHS = dict(PATHS, objective_only=(1, 0, 1),
                  # and the y / z passes fused but not the objective: the
                  # inverse x pass then adds the gather's partial copies
                  fused_yz_only=(1, 1, 0))


def engine_on_path(w, dtype, path):
    t = tof()
    e = t.engine_for(w, dtype)
    zsum, fuse, fobj = GRAD_PATHS[path]
    e.set_option(t.OPT_ZSUM, zsum)
    e.set_option(t.OPT_FUSE_YZ, fuse)
    e.set_option(t.OPT_FUSE_OBJECTIVE, fobj)
    return e


_ORACLE = {}


def cached(key, fn):
    """Oracle results shared by the parametrizations of one case."""
    if key not in _ORACLE:
        _ORACLE[key] = fn()
    return _ORACLE[key]


# ---------------------------------------------------------------- tensor setup
@pytest.mark.parametrize("n,h", [((12, 10, 14), (1.0, 1.0, 1.0)), ((9, 11, 8), (0.7, 1.3, 0.9)),
                                 ((64, 64, 64), (1.0, 1.0, 0.5))])
def test_gpu_tensor_matches_oracle(torch, n, h):
    say("tensor", n, h)
    e = tof().Engine(n, h, "f64")
    N = host(e.tensor())
    ref = oracle.newell_table(n, h)
    for c in range(6):
        scale = np.abs(ref[c]).max()
        assert np.abs(N[c] - ref[c]).max() <= 1e-15 * scale, c


def masked(w, seed, fraction=0.6):
    """w with a seeded random design mask."""
    return dataclasses.replace(w, mask=wl.random_mask(seed, w.n, fraction))


def test_gpu_tensor_full_matches_oracle_at_signed_offsets(torch):
    """tof_tensor_full: every signed offset, against the oracle's octant with
    the parity signs (oracle.tensor_at), and the symmetry N(-k) = N(k)."""
    n, h = (7, 6, 5), (1.0, 0.8, 1.3)
    e = tof().Engine(n, h, "f64")
    F = host(e.tensor_full())
    assert F.shape == (6, 9, 11, 13)
    table = oracle.newell_table(n, h)
    comps = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    scale = np.abs(table).max()
    for kz in range(-4, 5):
        for ky in range(-5, 6):
            for kx in range(-6, 7):
                ref = oracle.tensor_at(table, (kx, ky, kz))
                got = F[:, kz + 4, ky + 5, kx + 6]
                for c, (a, b) in enumerate(comps):
                    assert abs(got[c] - ref[a, b]) <= 1e-15 * scale, (c, kx, ky, kz)
    # N(-k) = N(k); exact but for the rounding noise of the odd components on
    # their zero planes (k_a = 0), whose sign the parity flips
    assert np.abs(F - F[:, ::-1, ::-1, ::-1]).max() <= 2e-15 * scale


# ---------------------------------------------------------------- field
FIELD_CASES = [
    ("c1", lambda: wl.config1()),
    ("ragged", lambda: wl.small_random(21, n=(13, 10, 7), h=(1.0, 0.8, 1.3))),
    ("vector_m0", lambda: wl.small_random(22, n=(9, 12, 10), varying_m0=True)),
    ("tilted_m0", lambda: wl.small_random(23, n=(10, 9, 11), m0=(0.3, -0.4, 0.866))),
    ("nonsmooth", lambda: wl.small_random(24, n=(11, 13, 6), h=(1.0, 1.0, 1.0))),  # 2n = 22, 26: L = 24, 28
    # two design rows, Ly = 32: the few-source-row paths
    ("thin_design", lambda: wl.small_random(25, n=(11, 16, 9), design=(1, 10, 0, 16, 2, 4))),
    # a random design mask inside the box (chi = box and mask)
    ("masked", lambda: masked(wl.small_random(27, n=(12, 11, 10), design=(1, 11, 0, 11, 0, 7)), 27)),
]


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make", FIELD_CASES)
def test_gpu_field_matches_direct_sum(torch, name, make, dtype, path):
    w = make()
    say("field", name, dtype, path, w.n)
    e = engine_on_path(w, dtype, path)
    tdt = e.dtype
    H = host(e.field(dev(torch, w.rho, tdt), comps=7))
    torch.cuda.synchronize()
    nx, ny, nz = w.n
    ref = cached(("field", name), lambda: oracle.field(w.n, w.h, oracle.magnetization(w), w.design,
                                                       (0, nx, 0, ny, 0, nz), oracle.m0_mask(w), 7))
    assert rel_inf(H, ref) <= TOL[dtype], rel_inf(H, ref)
    # single components in component order
    Hz = host(e.field(dev(torch, w.rho, tdt), comps=4))
    assert rel_inf(Hz[0], ref[2]) <= TOL[dtype]
    Hxz = host(e.field(dev(torch, w.rho, tdt), comps=5))
    assert rel_inf(Hxz, ref[[0, 2]]) <= TOL[dtype]


# ---------------------------------------------------------------- gradient
GRAD_CASES = [
    ("c1", lambda: wl.config1()),
    ("c2", lambda: wl.config2()),
    ("gradxy_ragged", lambda: wl.small_random(31, n=(17, 13, 11), h=(0.7, 1.3, 0.9))),
    ("p4", lambda: wl.small_random(32, n=(12, 14, 9), p=4)),
    ("htarget_vector", lambda: wl.small_random(33, n=(10, 11, 12), j_kind=wl.J_MEAN_SQ_H_TARGET,
                                               varying_m0=True)),
    ("neg_half_tilted", lambda: wl.small_random(34, n=(9, 10, 8), j_kind=wl.J_NEG_HALF_HZ2,
                                                m0=(0.3, -0.4, 0.866))),
    ("mean_sq_hz_corner", lambda: wl.small_random(35, n=(8, 8, 9), j_kind=wl.J_MEAN_SQ_HZ,
                                                  sensor=(0, 3, 5, 8, 8, 9))),
    ("p1_single_design_cell", lambda: wl.small_random(36, n=(7, 6, 8), p=1, design=(3, 4, 2, 3, 1, 2))),
    # three sensor rows with Ly = 32: the fused kernels' multi-row variants
    ("sensor3_pow2y", lambda: wl.small_random(37, n=(19, 16, 13), sensor=(6, 12, 5, 11, 10, 13))),
    # varying M0 and a vector target with Ly = 64: three components in and out
    ("vector_pow2y", lambda: wl.small_random(38, n=(12, 32, 10), j_kind=wl.J_MEAN_SQ_H_TARGET, varying_m0=True)),
    # field and gradient objective (strip on three sides), Lx = Ly = 32, non-cubic cells
    ("field_gradient", lambda: wl.small_random(39, n=(14, 16, 10), h=(0.8, 1.2, 1.0), j_kind=wl.J_FIELD_GRADIENT)),
    ("field_gradient_ragged", lambda: wl.small_random(40, n=(13, 11, 9), j_kind=wl.J_FIELD_GRADIENT)),
    # two design layers and Lx = Ly = 32: on the fused path the adjoint's
    # target has few rows (the gather), so J is formed by a kernel of its own
    ("thin_design_grad", lambda: wl.small_random(26, n=(16, 16, 9), design=(0, 16, 0, 16, 2, 4))),
    # random design masks: the uniform-M0 Hz objective (Ly = 32: fused kernels) and
    # varying M0 with a vector target (three components through the masked epilogue)
    ("masked_gradxy", lambda: masked(wl.small_random(44, n=(16, 16, 11), design=(0, 16, 0, 16, 0, 7)), 44)),
    ("masked_vector", lambda: masked(wl.small_random(45, n=(10, 12, 9), j_kind=wl.J_MEAN_SQ_H_TARGET,
                                                     varying_m0=True), 45, 0.5)),
    # Lx = Ly = 32 for 13 x 11 cells: rows in the lower half of the padded
    # lines without filling it (the forward x pass's and the gather's bounded
    # lower-half forms), with the design box at the origin and offset in x and y
    ("lower_half_rows", lambda: dataclasses.replace(wl.small_random(46, n=(13, 11, 10)), pad=(32, 32, 20))),
    ("lower_half_offset_design", lambda: dataclasses.replace(
        wl.small_random(47, n=(13, 11, 10), design=(2, 12, 3, 10, 0, 6)), pad=(32, 32, 20))),
    # the same with varying M0 and a vector target: three components through
    # the lower-half forms of the x pass and the gather
    ("lower_half_vector", lambda: dataclasses.replace(
        wl.small_random(48, n=(13, 11, 10), j_kind=wl.J_MEAN_SQ_H_TARGET, varying_m0=True), pad=(32, 32, 20))),
]


@pytest.mark.parametrize("path", list(GRAD_PATHS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make", GRAD_CASES)
def test_gpu_objective_and_grad_match_oracle(torch, name, make, dtype, path):
    w = make()
    say("grad", name, dtype, path, w.n)
    e = engine_on_path(w, dtype, path)
    J, g = e.objective_and_grad(dev(torch, w.rho, e.dtype))
    torch.cuda.synchronize()
    J = float(J.item())
    g = host(g)
    Jr, gr, _ = cached(("grad", name), lambda: oracle.objective_and_grad(w))
    assert abs(J - Jr) <= TOL[dtype] * abs(Jr), (J, Jr)
    assert rel_inf(g, gr) <= TOL[dtype], rel_inf(g, gr)
    # zero outside the design region (box and mask)
    chi = oracle.design_chi(w)
    assert np.all(g[chi == 0] == 0.0)


@pytest.mark.parametrize("path", list(GRAD_PATHS))
def test_gpu_objective_and_grad_without_J(torch, path):
    """J is optional at the boundary: with a NULL J the gradient is the same,
    bit for bit, on every path (nothing forms or writes J)."""
    t = tof()
    w = wl.small_random(43, n=(16, 16, 9))
    say("grad without J", path, w.n)
    e = engine_on_path(w, "f32", path)
    rho = dev(torch, w.rho, e.dtype)
    J, g_ref = e.objective_and_grad(rho)
    g = torch.full_like(g_ref, float("nan"))
    st = t.lib().tof_objective_and_grad(e._ctx, ctypes.c_void_p(rho.data_ptr()), None,
                                        ctypes.c_void_p(g.data_ptr()), None)
    torch.cuda.synchronize()
    assert st == 0, t.lib().tof_last_error(e._ctx)
    assert torch.equal(g, g_ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gpu_adjoint_vjp_matches_oracle(torch, dtype):
    w = wl.small_random(41, n=(11, 9, 10), varying_m0=True)
    say("adjoint", dtype)
    e = tof().engine_for(w, dtype)
    rng = np.random.default_rng(5)
    gH = rng.normal(size=(3,) + w.rho.shape)
    grad = host(e.adjoint(dev(torch, w.rho, e.dtype), dev(torch, gH, e.dtype)))
    nx, ny, nz = w.n
    A = oracle.field(w.n, w.h, gH, (0, nx, 0, ny, 0, nz), w.design, 7, 7)
    ref = oracle.gradient_from_adjoint(w, A)
    assert rel_inf(grad, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gpu_c2_hundred_evaluations(torch, dtype):
    """Configuration 2 as specified: 100 gradient evaluations of the
    64 x 64 x 64 problem.  Every J equals the first bit for bit (fixed-order
    reductions), so does the last gradient, and both match the oracle."""
    w = wl.config2()
    e = tof().engine_for(w, dtype)
    rho = dev(torch, w.rho, e.dtype)
    J0, g0 = e.objective_and_grad(rho)
    g = torch.empty_like(g0)
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    Js = torch.empty(100, dtype=torch.float64, device="cuda")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for k in range(100):
        e.objective_and_grad(rho, g, J)
        Js[k:k + 1].copy_(J)
    t1.record()
    torch.cuda.synchronize()
    say(f"c2 {dtype}: 100 evaluations, {t0.elapsed_time(t1) / 100:.4f} ms each (with the J copies)")
    assert torch.all(Js == J0)
    assert torch.equal(g, g0)
    Jr, gr, _ = cached(("grad", "c2"), lambda: oracle.objective_and_grad(w))
    assert abs(float(J0.item()) - Jr) <= TOL[dtype] * abs(Jr)
    assert rel_inf(host(g), gr) <= TOL[dtype]


def test_gpu_is_deterministic_and_stream_safe(torch):
    w = wl.config2()
    e = tof().engine_for(w, "f32")
    rho = dev(torch, w.rho, torch.float32)
    J1, g1 = e.objective_and_grad(rho)
    s = torch.cuda.Stream()
    # calls on one context must not overlap: the side stream waits for the first call
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        J2, g2 = e.objective_and_grad(rho)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(J1, J2)


STEP_TOL = {"f64": 1e-15, "f32": 2.5e-7}   # rho in [0, 1]: a few ulp of 1


@pytest.mark.parametrize("with_mask", [False, True])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gpu_project_step_matches_oracle(torch, dtype, with_mask):
    """tof_project_step against the oracle's projected step, on the same
    density and gradient (the gradient of the problem itself), with and
    without a design mask; cells outside chi keep their value exactly."""
    w = wl.small_random(42, n=(10, 9, 8), design=(1, 9, 0, 8, 0, 6))
    if with_mask:
        w = masked(w, 42)
    say("project step", dtype, with_mask)
    e = tof().engine_for(w, dtype)
    rho = dev(torch, w.rho, e.dtype)
    rho0 = host(rho)
    J, g = e.objective_and_grad(rho)
    gh = host(g)
    e.project_step(rho, g, 0.05)
    torch.cuda.synchronize()
    got = host(rho)
    want = oracle.project_step(w, rho0, gh, 0.05)
    assert np.abs(got - want).max() <= STEP_TOL[dtype]
    chi = oracle.design_chi(w)
    assert np.array_equal(got[chi == 0], rho0[chi == 0])
    # clamping at both bounds: a large step along a gradient of both signs
    # drives cells to 0 and to 1
    flip = np.where(np.random.default_rng(7).random(gh.shape) < 0.5, -1.0, 1.0)
    gmix = dev(torch, gh * flip, e.dtype)
    e.project_step(rho, gmix, 5.0)
    torch.cuda.synchronize()
    got2 = host(rho)
    want2 = oracle.project_step(w, got, host(gmix), 5.0)
    assert np.abs(got2 - want2).max() <= STEP_TOL[dtype]
    assert np.any(got2[chi == 1] == 0.0) and np.any(got2[chi == 1] == 1.0)


def test_gpu_project_step_zero_gradient(torch):
    """G = 0 leaves rho unchanged, also values outside [0, 1]."""
    w = wl.small_random(46, n=(8, 7, 6))
    e = tof().engine_for(w, "f64")
    r = w.rho.copy()
    r[0, 0, 0], r[1, 2, 3] = 1.5, -0.25
    rho = dev(torch, r, torch.float64)
    e.project_step(rho, torch.zeros_like(rho), 0.3)
    torch.cuda.synchronize()
    assert np.array_equal(host(rho), r)


def test_gpu_zero_density(torch):
    w = wl.config1()
    w = dataclasses.replace(w, rho=np.zeros_like(w.rho))
    e = tof().engine_for(w, "f32")
    J, g = e.objective_and_grad(dev(torch, w.rho, torch.float32))
    torch.cuda.synchronize()
    assert abs(J.item() - 0.01) < 1e-15
    assert torch.count_nonzero(g).item() == 0


# ---------------------------------------------------------------- full size
def c3_reference(cache):
    """The oracle's J and full gradient of the 256 x 256 x 128 workload
    (direct sums over every design cell; computed once per test run)."""
    if "c3" not in cache:
        w = wl.config3()
        say(f"oracle: full 256x256x128 gradient on {oracle.num_threads()} threads ...")
        t0 = time.perf_counter()
        J, g, _ = oracle.objective_and_grad(w)
        say(f"  oracle done in {time.perf_counter() - t0:.1f} s")
        cache["c3"] = (J, g)
    return cache["c3"]


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_gpu_full_size_256x256x128(torch, oracle_cache, dtype, path):
    """The benchmark workload (256 x 256 x 128, padded 512 x 512 x 256) on
    each pass choice (fused: the benchmark's launch configuration; the direct
    z sum in its own pass; FFTs along z with Lz = 256): J and the whole
    gradient array against the oracle's direct sums."""
    w = wl.config3()
    say("full size", dtype, path)
    e = engine_on_path(w, dtype, path)
    assert e.padded_lengths() == (512, 512, 256)
    J, g = e.objective_and_grad(dev(torch, w.rho, e.dtype))
    torch.cuda.synchronize()
    g = host(g)
    e.close()
    Jr, gr = c3_reference(oracle_cache)
    err = rel_inf(g, gr)
    say(f"  rel err J {abs(float(J.item()) - Jr) / abs(Jr):.2e}, grad {err:.2e}")
    assert abs(float(J.item()) - Jr) <= TOL[dtype] * abs(Jr)
    assert err <= TOL[dtype]
    assert np.all(g[124:] == 0.0)


# ---------------------------------------------------------------- boundary
def test_gpu_validate_rejects_non_finite_inputs(torch):
    """With validation on, NaN or infinite inputs return TOF_ERR_INVALID
    before anything else is launched (the outputs stay untouched); finite
    inputs give the same result as without validation."""
    t = tof()
    w = wl.small_random(47, n=(12, 10, 9))
    ev = t.engine_for(w, "f32", validate=True)
    e = t.engine_for(w, "f32")
    rho = dev(torch, w.rho, torch.float32)
    Jv, gv = ev.objective_and_grad(rho)
    J, g = e.objective_and_grad(rho)
    torch.cuda.synchronize()
    assert torch.equal(gv, g) and torch.equal(Jv, J)
    for bad in (float("nan"), float("inf"), -float("inf")):
        r = rho.clone()
        r[3, 4, 5] = bad
        out = torch.full_like(rho, 7.0)
        with pytest.raises(t.TofError) as ei:
            ev.objective_and_grad(r, out)
        assert ei.value.status == -1 and "rho" in str(ei.value)
        with pytest.raises(t.TofError):
            ev.field(r)
        torch.cuda.synchronize()
        assert torch.all(out == 7.0)
    gH = torch.zeros((3,) + rho.shape, dtype=torch.float32, device="cuda")
    gH[1, 2, 3, 4] = float("nan")
    with pytest.raises(t.TofError) as ei:
        ev.adjoint(rho, gH)
    assert "gH" in str(ei.value)
    # without validation the call goes through (NaN propagates)
    r = rho.clone()
    r[3, 4, 5] = float("nan")
    J2, g2 = e.objective_and_grad(r)
    torch.cuda.synchronize()
    assert torch.isnan(J2).any() or torch.isnan(g2).any()


def test_gpu_tensor_trace_self_check(torch):
    """Setup checks max |tr N(k) - delta_k0| < 1e-12; the test hook that adds
    1e-9 to one tensor entry makes tof_create fail with TOF_ERR_NUMERIC."""
    t = tof()
    t.Engine((9, 8, 7), (1.0, 0.8, 1.3), "f64").close()
    with pytest.raises(t.TofError) as ei:
        t.Engine((9, 8, 7), (1.0, 0.8, 1.3), "f64", flags=t.GRID_SELFTEST_PERTURB)
    assert ei.value.status == -5 and "trace" in str(ei.value)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_gpu_workspace_bytes_before_create_match_the_context(torch, dtype):
    t = tof()
    for n, L in (((256, 256, 128), None), ((13, 10, 7), None), ((16, 16, 9), (32, 32, 32))):
        want = t.workspace_bytes(n, (1.0, 1.0, 1.0), dtype, L)
        e = t.Engine(n, (1.0, 1.0, 1.0), dtype, L=L)
        assert e.ctx_bytes() == want, (n, L)
        e.close()


def test_gpu_device_target_field_equals_host(torch):
    """Kind 3 with H* given as a device pointer gives the same result, bit
    for bit, as with H* from host memory."""
    t = tof()
    w = wl.small_random(48, n=(10, 11, 12), j_kind=wl.J_MEAN_SQ_H_TARGET, varying_m0=True)
    e = t.engine_for(w, "f64")
    rho = dev(torch, w.rho, torch.float64)
    J1, g1 = e.objective_and_grad(rho)
    J1, g1 = J1.clone(), g1.clone()
    e.set_objective(w.j_kind, w.sensor, w.j_target, w.j_lambda, dev(torch, w.h_target, torch.float64))
    J2, g2 = e.objective_and_grad(rho)
    torch.cuda.synchronize()
    assert torch.equal(J1, J2) and torch.equal(g1, g2)
    # a rejected objective (sensor outside the grid) leaves the previous one in place
    with pytest.raises(t.TofError):
        e.set_objective(w.j_kind, (0, 99, 0, 2, 0, 1), 0.0, 0.0, w.h_target)
    J3, g3 = e.objective_and_grad(rho)
    torch.cuda.synchronize()
    assert torch.equal(J1, J3) and torch.equal(g1, g3)


# ---------------------------------------------------------------- tile options, graphs
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_gpu_tile_options_do_not_change_the_result(torch, dtype):
    """The x tile and the scatter's row groups change only the work split:
    the gradient is the same bit for bit; the gather's row groups change the
    order of its partial sums, so the gradient agrees to rounding."""
    t = tof()
    w = wl.small_random(49, n=(40, 48, 19), design=(0, 40, 0, 48, 0, 15), sensor=(12, 28, 14, 34, 18, 19))
    e = t.engine_for(w, dtype, L=(128, 128, 40))
    rho = dev(torch, w.rho, e.dtype)
    J0, g0 = e.objective_and_grad(rho)
    J0, g0 = J0.clone(), g0.clone()
    for opt, vals in ((t.OPT_X_TILE, (1, 2, 0)), (t.OPT_SCATTER_GROUPS, (1, 3, 7, 0))):
        for v in vals:
            e.set_option(opt, v)
            J, g = e.objective_and_grad(rho)
            torch.cuda.synchronize()
            assert torch.equal(g, g0) and torch.equal(J, J0), (opt, v)
    for v in (1, 2, 5):
        e.set_option(t.OPT_GATHER_GROUPS, v)
        J, g = e.objective_and_grad(rho)
        torch.cuda.synchronize()
        tol = 1e-12 if dtype == "f64" else 2e-6
        assert abs(J.item() - J0.item()) <= tol * abs(J0.item())
        assert float((g - g0).abs().max()) <= tol * float(g0.abs().max())
    with pytest.raises(t.TofError):
        e.set_option(t.OPT_X_TILE, 3)
    with pytest.raises(t.TofError):
        e.set_option(t.OPT_GATHER_GROUPS, 65)


def test_gpu_graph_replays_of_one_evaluation(torch):
    """One gradient evaluation recorded into a graph: three replays, with
    the program's own eager work and synchronizations between them, each
    equal bit for bit to the eager evaluation (the hot calls record no
    memset or host synchronization)."""
    t = tof()
    w = wl.config2()
    e = t.engine_for(w, "f32")
    rho = dev(torch, w.rho, torch.float32)
    J_ref, g_ref = e.objective_and_grad(rho)
    J_ref, g_ref = J_ref.clone(), g_ref.clone()
    g = torch.empty_like(rho)
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        e.objective_and_grad(rho, g, J, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for k in range(3):
        g.fill_(float("nan"))
        J.fill_(float("nan"))
        x = torch.randn(1 << 20, device="cuda")
        (x * 3).sum().item()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref) and torch.equal(J, J_ref), k


def test_gpu_profile_launch_times_add_up_to_the_step(torch):
    """Per-launch timing over consecutive evaluations: with an event per
    launch, every launch after the first is timed from the end of the one
    before it, so the slots' means add up to one evaluation as it runs with
    those events (each launch a little longer: between 0.9 and 1.3 times
    the plain step) and every slot of the fused path counts one launch per
    evaluation (the chain's first launch aside).  Bursts (each pass again
    back to back, events around the burst only) add up to the plain step
    within 15%, and leave the evaluation's results bit for bit unchanged."""
    w = wl.config3()
    e = tof().engine_for(w, "f32")
    rho = torch.as_tensor(w.rho, dtype=e.dtype, device="cuda")
    grad = torch.empty_like(rho)
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    for _ in range(20):
        e.objective_and_grad(rho, grad, J)
    n = 100

    def step_ms():
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(n):
            e.objective_and_grad(rho, grad, J)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / n

    step = sorted(step_ms() for _ in range(3))[1]
    g0, J0 = grad.clone(), J.clone()
    e.profile(True)
    for _ in range(n):
        e.objective_and_grad(rho, grad, J)
    prof = e.profile_read()
    used = [(i, name, ms, cnt) for i, (name, ms, cnt, _) in enumerate(prof) if cnt > 0]
    bursts = []
    for _ in range(3):
        e.profile_burst([i for (i, _, _, _) in used], 50)
        grad.fill_(float("nan"))
        e.objective_and_grad(rho, grad, J)
        bursts.append(e.profile_burst_read())
        assert torch.equal(grad, g0) and torch.equal(J, J0)
    e.profile_read()
    e.profile(False)
    burst = [sorted(b[i] for b in bursts)[1] for i in range(len(bursts[0]))]
    say("step", step, "event per launch", [(name, round(ms / cnt * 1e3, 2), cnt) for (_, name, ms, cnt) in used],
        "bursts", [(name, round(burst[i] * 1e3, 2)) for (i, name, _, _) in used])
    assert len(used) == 5
    assert sorted(cnt for (_, _, _, cnt) in used) == [n - 1, n, n, n, n]
    total = sum(ms / cnt for (_, _, ms, cnt) in used)
    assert 0.9 * step <= total <= 1.3 * step, (total, step)
    assert all(burst[i] > 0 for (i, _, _, _) in used)
    btotal = sum(burst[i] for (i, _, _, _) in used)
    assert 0.9 * step <= btotal <= 1.15 * step, (btotal, step)
    e.close()


def test_gpu_profile_burst_rejects_bad_arguments(torch):
    """tof_profile_burst: refused with timing off, repeats outside [1, 4096]
    and a mask naming no slot; tof_profile_burst_read refuses a null array."""
    t = tof()
    L = t.lib()
    e = t.Engine((8, 8, 8), (1.0, 1.0, 1.0), "f32")
    assert L.tof_profile_burst(e._ctx, 1, 10) == -1          # timing off
    e.profile(True)
    assert L.tof_profile_burst(e._ctx, 1, 0) == -1
    assert L.tof_profile_burst(e._ctx, 1, 4097) == -1
    assert L.tof_profile_burst(e._ctx, 1 << 12, 10) == -1    # TOF_PROFILE_SLOTS = 12
    assert L.tof_profile_burst(e._ctx, 1, 4096) == 0
    assert L.tof_profile_burst_read(e._ctx, None) == -1
    e.profile(False)
    e.close()
