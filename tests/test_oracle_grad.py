"""Pins of the oracle's objective and adjoint gradient (Sec. Methodology,
eqs. (dj_drho), (adjoint1), (adjoint2)) against finite differences of J,
closed-form objectives and special cases.  The finite-difference tests fix the
sign of the gradient, which the paper prints with the opposite sign."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1707_09898_amd import workloads as wl


def fd_gradient(w, cells, step=1e-6, table=None):
    table = oracle.table_for(w) if table is None else table
    out = []
    for (z, y, x) in cells:
        vals = []
        for s in (+1.0, -1.0):
            r = w.rho.copy()
            r[z, y, x] += s * step
            H = oracle.forward_field(w, r, table=table)
            vals.append(oracle.objective(w, H)[0])
        out.append((vals[0] - vals[1]) / (2 * step))
    return np.array(out)


def design_cells(w, count, seed):
    rng = np.random.default_rng(seed)
    x0, x1, y0, y1, z0, z1 = w.design
    return [(int(rng.integers(z0, z1)), int(rng.integers(y0, y1)), int(rng.integers(x0, x1)))
            for _ in range(count)]


@pytest.mark.parametrize("make", [
    wl.config1,
    lambda: wl.small_random(11, n=(12, 10, 14)),
    lambda: wl.small_random(12, n=(9, 11, 8), h=(0.7, 1.3, 0.9), p=4),
    lambda: wl.small_random(13, n=(8, 8, 10), j_kind=wl.J_MEAN_SQ_H_TARGET, varying_m0=True),
    lambda: wl.small_random(14, n=(10, 9, 8), j_kind=wl.J_NEG_HALF_HZ2, m0=(0.3, -0.4, 0.866)),
    lambda: wl.small_random(15, n=(12, 11, 8), h=(0.8, 1.1, 1.0), j_kind=wl.J_FIELD_GRADIENT),
])
def test_gradient_matches_central_differences(make):
    w = make()
    table = oracle.table_for(w)
    J, grad, _ = oracle.objective_and_grad(w, table=table)
    cells = design_cells(w, 24, 0)
    fd = fd_gradient(w, cells, table=table)
    got = np.array([grad[c] for c in cells])
    scale = np.abs(grad).max()
    # FD truncation ~ step^2 |J'''|, rounding ~ eps |J| / step
    tol = 1e-6 * scale + 20 * 2.2e-16 * max(abs(J), 1e-30) / 1e-6
    assert np.abs(got - fd).max() <= tol, (np.abs(got - fd).max(), tol)
    # every sign agrees where the gradient is not tiny
    big = np.abs(fd) > 1e-3 * scale
    assert np.all(np.sign(got[big]) == np.sign(fd[big]))


def test_single_cell_gradient_sign():
    """One cubic cell, J = -1/2 V H_z^2: H_z = -rho^p/3, so J = -rho^(2p) V/18
    and dJ/drho = -p rho^(2p-1) V/9 (negative: more material, larger |H_z|)."""
    rho = np.array([[[0.7]]])
    w = wl.Workload(name="one", n=(1, 1, 1), h=(1.0, 1.0, 1.0), design=(0, 1, 0, 1, 0, 1),
                    sensor=(0, 1, 0, 1, 0, 1), p=3, rho=rho, j_kind=wl.J_NEG_HALF_HZ2)
    J, grad, H = oracle.objective_and_grad(w)
    assert abs(H[2, 0, 0, 0] + 0.7 ** 3 / 3) < 1e-16
    assert abs(J + 0.7 ** 6 / 18) < 1e-16
    assert abs(grad[0, 0, 0] + 3 * 0.7 ** 5 / 9) < 1e-16


def test_zero_density_gives_zero_field_and_gradient():
    w = wl.config1()
    w = dataclasses.replace(w, rho=np.zeros_like(w.rho))
    J, grad, H = oracle.objective_and_grad(w)
    assert np.all(H == 0.0)
    assert abs(J - 0.01) < 1e-17        # mean (0 - 0.1)^2
    assert np.all(grad == 0.0)          # p rho^(p-1) = 0 for p > 1


def test_uniform_density_scaling_law():
    """rho = c everywhere: H scales as c^p; for J = -1/2 V sum H_z^2 the
    gradient scales as c^(2p-1)."""
    base = wl.small_random(5, n=(8, 7, 9), j_kind=wl.J_NEG_HALF_HZ2)
    out = []
    for c in (0.5, 0.8):
        w = dataclasses.replace(base, rho=np.full_like(base.rho, c))
        J, grad, H = oracle.objective_and_grad(w)
        out.append((H, grad))
    (H1, g1), (H2, g2) = out
    r = 0.8 / 0.5
    np.testing.assert_allclose(H2, H1 * r ** 3, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(g2, g1 * r ** 5, rtol=1e-12, atol=1e-300)


def _field_workload(kind):
    w = wl.small_random(3, n=(10, 9, 6), j_kind=kind)
    return w


def test_objective_constant_field():
    """H_z = c on every cell: the difference terms vanish, J = (c - t)^2."""
    w = _field_workload(wl.J_MEAN_SQ_HZ_GRADXY)
    H = np.zeros((3, 6, 9, 10))
    H[2] = 0.35
    J, g = oracle.objective(w, H)
    assert abs(J - (0.35 - 0.2) ** 2) < 1e-16


def test_objective_linear_field():
    """H_z = a + b x + c y: central differences are exact, D_x = b/dx-units,
    so J = mean (H_z - t)^2 + lam (b^2 + c^2) with b, c per unit length."""
    w = dataclasses.replace(_field_workload(wl.J_MEAN_SQ_HZ_GRADXY), h=(0.5, 2.0, 1.0))
    nz, ny, nx = 6, 9, 10
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c = 0.1, 0.03, -0.02     # per cell
    H = np.zeros((3, nz, ny, nx))
    H[2] = a + b * x + c * y
    J, g = oracle.objective(w, H)
    x0, x1, y0, y1, z0, z1 = w.sensor
    d = H[2, z0:z1, y0:y1, x0:x1] - 0.2
    want = float(np.mean(d * d)) + 0.01 * ((b / 0.5) ** 2 + (c / 2.0) ** 2)
    assert abs(J - want) < 1e-15


def test_objective_gradient_is_exact_derivative():
    """g = dJ/dH checked by central differences of J in H (J is quadratic in
    H, so central differences are exact up to rounding)."""
    rng = np.random.default_rng(4)
    for kind in (wl.J_MEAN_SQ_HZ, wl.J_MEAN_SQ_HZ_GRADXY, wl.J_MEAN_SQ_H_TARGET, wl.J_NEG_HALF_HZ2,
                 wl.J_FIELD_GRADIENT):
        w = wl.small_random(8, n=(9, 8, 5), j_kind=kind)
        H = rng.normal(size=(3, 5, 8, 9)) * 0.1
        J, g = oracle.objective(w, H)
        for _ in range(30):
            idx = tuple(int(rng.integers(0, s)) for s in H.shape)
            Hp, Hm = H.copy(), H.copy()
            Hp[idx] += 1e-3
            Hm[idx] -= 1e-3
            fd = (oracle.objective(w, Hp)[0] - oracle.objective(w, Hm)[0]) / 2e-3
            assert abs(fd - g[idx]) < 1e-10 * max(1.0, abs(g).max())


def test_field_gradient_objective_linear_field():
    """Kind 5 with H_z = a + b x + c y (per cell): the forward differences
    along the strip's outward normals are exact (-b/dx on the -x side, +b/dx
    on the +x side, -c/dy on the -y side), so J has a closed form."""
    w = dataclasses.replace(wl.small_random(3, n=(12, 11, 6), j_kind=wl.J_FIELD_GRADIENT), h=(0.5, 2.0, 1.0))
    nz, ny, nx = 6, 11, 12
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c = 0.1, 0.03, -0.02
    H = np.zeros((3, nz, ny, nx))
    H[2] = a + b * x + c * y
    J, g = oracle.objective(w, H)
    x0, x1, y0, y1, z0, z1 = w.sensor
    V = 0.5 * 2.0 * 1.0
    field = H[2, z0:z1, y0:y1, x0:x1]
    strip = (z1 - z0) * ((y1 - y0) * 2 * (b / 0.5) ** 2 + (x1 - x0) * (c / 2.0) ** 2)
    want = -0.5 * V * (float(np.sum(field * field)) + w.j_lambda * strip)
    assert abs(J - want) <= 1e-15 * abs(want)


def test_field_gradient_objective_derivative_on_every_cell():
    """Kind 5: g = dJ/dH_z by central differences at every cell of the
    objective box (field, strip and the strip's outer neighbours)."""
    rng = np.random.default_rng(6)
    w = wl.small_random(9, n=(12, 11, 5), j_kind=wl.J_FIELD_GRADIENT)
    H = rng.normal(size=(3, 5, 11, 12)) * 0.1
    J, g = oracle.objective(w, H)
    x0, x1, y0, y1, z0, z1 = oracle.objective_box(w)
    nonzero = 0
    for zz in range(z0, z1):
        for yy in range(y0, y1):
            for xx in range(x0, x1):
                Hp, Hm = H.copy(), H.copy()
                Hp[2, zz, yy, xx] += 1e-3
                Hm[2, zz, yy, xx] -= 1e-3
                fd = (oracle.objective(w, Hp)[0] - oracle.objective(w, Hm)[0]) / 2e-3
                assert abs(fd - g[2, zz, yy, xx]) < 1e-12 * max(1.0, abs(g).max())
                nonzero += g[2, zz, yy, xx] != 0
    # outside the field, the strip and its outer neighbours, J does not depend on H
    assert np.count_nonzero(g) == nonzero
