"""Pins of three oracle parts that the other oracle tests do not fix:

* objective kind 3, J = (1/S) sum_s |H_s - H*_s|^2 (the general J of
  eq. (objective_function) with a target field), by closed forms that a
  mis-normalization (1/(3S), a sum instead of a mean), a dropped component or
  a misaligned H* would fail;
* the projected-gradient update that keeps 0 <= rho <= 1 (the bound of
  Sec. Methodology, handled by the minimizer of Sec. Discretization), by a
  hand-computed case, its special cases and a descent property;
* the design mask (chi = box and mask), by reduction to the unmasked and to
  the single-cell-box problems, linearity of the field in the source, and
  central finite differences of J.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1707_09898_amd import workloads as wl


# ---------------------------------------------------------------- kind 3
def _kind3(n, sensor, h_target):
    rho = np.zeros((n[2], n[1], n[0]))
    return wl.Workload(name="k3", n=n, h=(1.0, 1.0, 1.0), design=(0, n[0], 0, n[1], 0, 1), sensor=sensor,
                       p=3, rho=rho, j_kind=wl.J_MEAN_SQ_H_TARGET, j_target=0.0, j_lambda=0.0,
                       h_target=h_target)


def test_kind3_one_cell_by_hand():
    """One sensor cell, H = (0.3, -0.2, 0.5), H* = (0.1, 0.1, 0.1):
    J = 0.2^2 + 0.3^2 + 0.4^2 = 0.29 and dJ/dH = 2 (H - H*) = (0.4, -0.6, 0.8)."""
    n = (3, 2, 4)
    ht = np.full((3, 1, 1, 1), 0.1)
    w = _kind3(n, (1, 2, 0, 1, 2, 3), ht)
    H = np.zeros((3, 4, 2, 3))
    H[:, 2, 0, 1] = (0.3, -0.2, 0.5)
    J, g = oracle.objective(w, H)
    assert abs(J - 0.29) < 1e-16
    assert np.allclose(g[:, 2, 0, 1], (0.4, -0.6, 0.8), rtol=0, atol=4e-16)
    g[:, 2, 0, 1] = 0.0
    assert np.all(g == 0.0)


def test_kind3_constant_difference_is_a_mean_over_cells_and_a_sum_over_components():
    """H = F + d on a 4 x 3 x 2 sensor box, H* = F with F varying per cell and
    per component, d constant: J = |d|^2 exactly (a mean over the 24 cells,
    a sum over the 3 components).  1/(3S) would give |d|^2/3, a sum over
    cells 24 |d|^2, Hz alone d_z^2, and an H* read in another cell order a
    value that depends on F."""
    n = (7, 6, 5)
    sensor = (2, 6, 1, 4, 3, 5)
    rng = np.random.default_rng(11)
    sshape = (2, 3, 4)
    F = rng.uniform(-1.0, 1.0, (3,) + sshape)
    d = np.array([0.05, -0.02, 0.03])
    w = _kind3(n, sensor, F)
    H = np.zeros((3, 5, 6, 7))
    x0, x1, y0, y1, z0, z1 = sensor
    H[:, z0:z1, y0:y1, x0:x1] = F + d[:, None, None, None]
    J, g = oracle.objective(w, H)
    assert abs(J - float(d @ d)) <= 4e-16 * float(d @ d) * 24
    assert np.allclose(g[:, z0:z1, y0:y1, x0:x1], (2.0 * d / 24)[:, None, None, None] * np.ones((3,) + sshape),
                       rtol=1e-12, atol=0)


def test_kind3_integer_pattern_closed_form():
    """H - H* = (1, 2, 3) q on the cell with C-order index q over the sensor
    box (q = 0 .. S-1): J = (1 + 4 + 9) / S * sum q^2 = 14 (S-1)(2S-1)/6."""
    n = (5, 4, 3)
    sensor = (0, 5, 1, 4, 1, 3)      # 5 x 3 x 2 = 30 cells
    S = 30
    q = np.arange(S, dtype=np.float64).reshape(2, 3, 5)
    ht = np.stack([np.full(q.shape, 0.25), np.full(q.shape, -0.5), np.full(q.shape, 1.0)])
    w = _kind3(n, sensor, ht)
    H = np.zeros((3, 3, 4, 5))
    H[:, 1:3, 1:4, 0:5] = ht + np.array([1.0, 2.0, 3.0])[:, None, None, None] * q
    J, _ = oracle.objective(w, H)
    want = 14.0 * (S - 1) * (2 * S - 1) / 6.0
    assert abs(J - want) <= 1e-14 * want


# ---------------------------------------------------------------- projected step
def _line(rho, grad_design_box=(0, 3, 0, 1, 0, 1), mask=None):
    n = (rho.shape[2], rho.shape[1], rho.shape[0])
    return wl.Workload(name="line", n=n, h=(1.0, 1.0, 1.0), design=grad_design_box, sensor=(0, 1, 0, 1, 0, 1),
                       p=3, rho=rho, mask=mask)


def test_project_step_three_cells_by_hand():
    """rho = (0.5, 0.02, 0.97), grad = (0.4, 2.0, -1.6), alpha = 0.05: the
    largest |grad| is 2, so rho - 0.025 grad = (0.49, -0.03, 1.01), clamped
    to (0.49, 0, 1): both bounds."""
    rho = np.array([[[0.5, 0.02, 0.97]]])
    grad = np.array([[[0.4, 2.0, -1.6]]])
    w = _line(rho)
    out = oracle.project_step(w, rho, grad, 0.05)
    assert np.allclose(out, [[[0.49, 0.0, 1.0]]], rtol=0, atol=4e-16)
    assert out[0, 0, 1] == 0.0 and out[0, 0, 2] == 1.0
    # the input is not modified
    assert rho[0, 0, 1] == 0.02


def test_project_step_zero_gradient_leaves_rho_unchanged():
    """G = 0: no step, not even the clamp (a value outside [0, 1] stays)."""
    rho = np.array([[[0.5, 1.5, -0.25]]])
    out = oracle.project_step(_line(rho), rho, np.zeros_like(rho), 0.3)
    assert np.array_equal(out, rho)


def test_project_step_only_moves_design_cells_and_normalizes_over_them():
    """Cells outside the design box keep their value, and a large gradient
    there does not enter G: design box x in [1, 3) of a 4-cell line."""
    rho = np.array([[[0.3, 0.6, 0.6, 0.9]]])
    grad = np.array([[[100.0, 1.0, -0.5, -100.0]]])
    w = _line(rho, grad_design_box=(1, 3, 0, 1, 0, 1))
    out = oracle.project_step(w, rho, grad, 0.1)
    assert np.allclose(out, [[[0.3, 0.5, 0.65, 0.9]]], rtol=0, atol=4e-16)


def test_project_step_respects_the_mask():
    """A masked-out cell of the design box is not moved and not counted in G."""
    rho = np.array([[[0.4, 0.4, 0.4]]])
    grad = np.array([[[1.0, 50.0, -2.0]]])
    mask = np.array([[[1, 0, 1]]], dtype=np.uint8)
    out = oracle.project_step(_line(rho, mask=mask), rho, grad, 0.2)
    assert np.allclose(out, [[[0.3, 0.4, 0.6]]], rtol=0, atol=4e-16)


def test_project_step_descends_on_a_real_objective():
    """With the true gradient and a small step, J decreases (the step is a
    descent direction scaled by 1/G > 0), and rho stays in [0, 1]."""
    w = wl.small_random(61, n=(9, 8, 7))
    table = oracle.table_for(w)
    J0, g, _ = oracle.objective_and_grad(w, table=table)
    rho1 = oracle.project_step(w, w.rho, g, 1e-3)
    J1, _, _ = oracle.objective_and_grad(w, rho1, table=table)
    assert J1 < J0
    assert rho1.min() >= 0.0 and rho1.max() <= 1.0
    # first-order prediction: J1 - J0 ~ -alpha/G sum g^2 on the unclamped cells
    G = np.abs(g).max()
    pred = -1e-3 / G * float(np.sum(g * g))
    assert abs((J1 - J0) - pred) <= 0.05 * abs(pred)


# ---------------------------------------------------------------- design mask
def test_mask_of_ones_is_no_mask():
    w = wl.small_random(62, n=(8, 9, 7))
    wm = dataclasses.replace(w, mask=np.ones_like(w.rho, dtype=np.uint8))
    J, g, H = oracle.objective_and_grad(w)
    Jm, gm, Hm = oracle.objective_and_grad(wm)
    assert J == Jm and np.array_equal(g, gm) and np.array_equal(H, Hm)


def test_mask_single_cell_equals_single_cell_design_box():
    """A whole-grid design box masked down to one cell is the problem whose
    design box is that cell: same field, J and gradient."""
    w = wl.small_random(63, n=(7, 6, 8), design=(2, 3, 4, 5, 1, 2))
    mask = np.zeros_like(w.rho, dtype=np.uint8)
    mask[1, 4, 2] = 1
    wm = dataclasses.replace(w, design=(0, 7, 0, 6, 0, 6), mask=mask)
    J, g, H = oracle.objective_and_grad(w)
    Jm, gm, Hm = oracle.objective_and_grad(wm)
    assert abs(J - Jm) <= 1e-15 * abs(J)
    assert np.abs(Hm - H).max() <= 1e-15 * np.abs(H).max()
    assert np.abs(gm - g).max() <= 1e-15 * np.abs(g).max()
    assert np.count_nonzero(gm) == 1 and gm[1, 4, 2] != 0.0


def test_mask_and_its_complement_add_up_to_the_box():
    """The field is linear in M: H(box and mask) + H(box and not mask) = H(box)."""
    w = wl.small_random(64, n=(9, 7, 8))
    mask = wl.random_mask(64, w.n, 0.6)
    nx, ny, nz = w.n
    whole = (0, nx, 0, ny, 0, nz)
    parts = []
    for m in (mask, 1 - mask, None):
        wm = dataclasses.replace(w, mask=m)
        parts.append(oracle.field(w.n, w.h, oracle.magnetization(wm), w.design, whole, 4, 7))
    a, b, c = parts
    assert np.abs(a + b - c).max() <= 1e-14 * np.abs(c).max()
    assert np.abs(a - c).max() > 1e-3 * np.abs(c).max()


@pytest.mark.parametrize("j_kind", [wl.J_MEAN_SQ_HZ_GRADXY, wl.J_MEAN_SQ_H_TARGET])
def test_masked_gradient_matches_central_differences(j_kind):
    """With a random mask, dJ/drho matches central differences on design
    cells and is exactly zero (as is the difference quotient) on masked-out
    cells of the box."""
    w = wl.small_random(65, n=(10, 9, 8), j_kind=j_kind, varying_m0=j_kind == wl.J_MEAN_SQ_H_TARGET)
    w = dataclasses.replace(w, mask=wl.random_mask(65, w.n, 0.5))
    table = oracle.table_for(w)
    J, grad, _ = oracle.objective_and_grad(w, table=table)
    chi = oracle.design_chi(w)
    rng = np.random.default_rng(9)
    x0, x1, y0, y1, z0, z1 = w.design
    cells = [(int(rng.integers(z0, z1)), int(rng.integers(y0, y1)), int(rng.integers(x0, x1))) for _ in range(24)]
    assert any(chi[c] == 0 for c in cells) and any(chi[c] == 1 for c in cells)
    scale = np.abs(grad).max()
    for c in cells:
        vals = []
        for s in (+1.0, -1.0):
            r = w.rho.copy()
            r[c] += s * 1e-6
            vals.append(oracle.objective(w, oracle.forward_field(w, r, table=table))[0])
        fd = (vals[0] - vals[1]) / 2e-6
        if chi[c] == 0:
            assert grad[c] == 0.0 and fd == 0.0
        else:
            assert abs(grad[c] - fd) <= 1e-6 * scale + 20 * 2.2e-16 * abs(J) / 1e-6
