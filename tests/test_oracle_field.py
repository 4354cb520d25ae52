"""Pins of the oracle's direct-sum stray field (eq. (convolution)), its adjoint
(the same operator, Sec. Methodology) and the zero-padded FFT formulation the
GPU path uses (Sec. Discretization: the FFT reaches the direct sum exactly)."""
import math

import numpy as np
import pytest

import oracle
from tests.test_oracle_tensor import aharoni_nz, dipole


def full_box(n):
    return (0, n[0], 0, n[1], 0, n[2])


def test_uniform_cube_mean_field_is_minus_one_third():
    """A fully magnetized cube of n^3 cubic cells: the mean of H_z over the cube
    is minus the self term of the aggregate cube, 1/3, for any n."""
    for n in (3, 5):
        N = (n, n, n)
        M = np.zeros((3, n, n, n))
        M[2] = 1.0
        H = oracle.field(N, (1.0, 1.0, 1.0), M, full_box(N), full_box(N), 4, 7)
        assert abs(H[2].mean() + 1.0 / 3.0) < 1e-14
        assert abs(H[0].mean()) < 1e-15 and abs(H[1].mean()) < 1e-15


def test_uniform_box_mean_field_matches_aharoni():
    """Mean field of a fully magnetized box of 4x3x5 cells of 1 x 1 x 0.5:
    -N_agg M with N_agg the prism's demagnetizing factor (Aharoni)."""
    n, h = (4, 3, 5), (1.0, 1.0, 0.5)
    for comp in range(3):
        M = np.zeros((3, n[2], n[1], n[0]))
        M[comp] = 1.0
        H = oracle.field(n, h, M, full_box(n), full_box(n), 1 << comp, 1 << comp)
        a, b, c = (n[i] * h[i] / 2 for i in range(3))
        want = [aharoni_nz(b, c, a), aharoni_nz(c, a, b), aharoni_nz(a, b, c)][comp]
        assert abs(H[comp].mean() + want) < 1e-14


def test_voxelized_sphere_field_is_minus_third_inside():
    """A uniformly magnetized sphere has H = -M/3 inside.  At the centre of a
    voxelized sphere the value is exact: the summed tensor is invariant under
    the cube's symmetry group, hence isotropic, and its trace is 1 (the
    self-term trace; every other offset has trace 0).  Elsewhere inside, the
    staircase surface leaves an error of a few 1e-3 at these radii."""
    for R in (4, 8, 12):
        n = 2 * R + 1
        c = np.arange(n) - R
        zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
        inside = (xx ** 2 + yy ** 2 + zz ** 2) <= R * R
        M = np.zeros((3, n, n, n))
        M[2][inside] = 1.0
        N = (n, n, n)
        q = R // 2
        tb = (R, R + q + 1, R, R + 1, R, R + q + 1)
        H = oracle.field(N, (1.0, 1.0, 1.0), M, full_box(N), tb, 4, 7)
        hc = H[:, R, R, R]
        assert abs(hc[0]) < 1e-15 and abs(hc[1]) < 1e-15
        assert abs(hc[2] + 1.0 / 3.0) < 1e-14
        if R >= 8:
            ho = H[:, R + q, R, R + q]
            assert np.abs(ho - np.array([0.0, 0.0, -1.0 / 3.0])).max() < 0.02


def test_single_cell_far_field_is_dipolar():
    n, h = (24, 20, 16), (1.0, 1.0, 0.5)
    M = np.zeros((3, n[2], n[1], n[0]))
    m = np.array([0.3, -0.5, 0.8])
    M[:, 0, 0, 0] = m
    tb = (20, 24, 16, 20, 12, 16)
    H = oracle.field(n, h, M, (0, 1, 0, 1, 0, 1), tb, 7, 7)
    V = h[0] * h[1] * h[2]
    t = (23, 19, 15)
    r = [t[a] * h[a] for a in range(3)]
    want = -dipole(r, V) @ m
    got = H[:, t[2], t[1], t[0]]
    assert np.abs(got - want).max() < 2e-3 * np.abs(want).max()


def test_linearity_and_translation_invariance():
    rng = np.random.default_rng(0)
    n, h = (9, 8, 7), (1.0, 0.8, 1.2)
    M1 = rng.normal(size=(3, 7, 8, 9))
    M2 = rng.normal(size=(3, 7, 8, 9))
    fb = full_box(n)
    H1 = oracle.field(n, h, M1, fb, fb)
    H2 = oracle.field(n, h, M2, fb, fb)
    H12 = oracle.field(n, h, 2.0 * M1 - 3.0 * M2, fb, fb)
    np.testing.assert_allclose(H12, 2.0 * H1 - 3.0 * H2, rtol=0, atol=1e-13 * np.abs(H12).max())
    # shift source and target boxes by the same vector
    sb, tb = (0, 4, 1, 5, 0, 3), (4, 8, 3, 6, 3, 6)
    Ha = oracle.field(n, h, M1, sb, tb)
    Ms = np.zeros_like(M1)
    Ms[:, 1:4, 2:6, 1:5] = M1[:, 0:3, 1:5, 0:4]
    Hb = oracle.field(n, h, Ms, (1, 5, 2, 6, 1, 4), (5, 9, 4, 7, 4, 7))
    np.testing.assert_allclose(Hb[:, 4:7, 4:7, 5:9], Ha[:, 3:6, 3:6, 4:8], rtol=0, atol=1e-15)


def wrapped_kernel(table, n, L):
    """Tensor wrapped onto the periodic box of lengths L (x, y, z): index i
    holds offset i for i < n and i - L for i > L - n; other slots zero."""
    out = np.zeros((3, 3, L[2], L[1], L[0]))
    for iz in range(L[2]):
        kz = iz if iz < n[2] else iz - L[2]
        if abs(kz) >= n[2]:
            continue
        for iy in range(L[1]):
            ky = iy if iy < n[1] else iy - L[1]
            if abs(ky) >= n[1]:
                continue
            for ix in range(L[0]):
                kx = ix if ix < n[0] else ix - L[0]
                if abs(kx) >= n[0]:
                    continue
                out[:, :, iz, iy, ix] = oracle.tensor_at(table, (kx, ky, kz))
    return out


@pytest.mark.parametrize("n,h,L", [((6, 5, 7), (1.0, 1.0, 1.0), (12, 10, 14)),
                                   ((5, 4, 6), (0.7, 1.3, 0.5), (9, 8, 11))])
def test_zero_padded_fft_convolution_equals_direct_sum(n, h, L):
    """The cyclic convolution on a box of L >= 2n - 1 cells per axis, with the
    source zero-padded, equals the linear one (the FFT route of Sec.
    Discretization).  numpy's FFT here is a test tool only."""
    rng = np.random.default_rng(1)
    nx, ny, nz = n
    M = rng.normal(size=(3, nz, ny, nx))
    table = oracle.newell_table(n, h)
    K = wrapped_kernel(table, n, L)
    Mp = np.zeros((3, L[2], L[1], L[0]))
    Mp[:, :nz, :ny, :nx] = M
    Mh = np.fft.fftn(Mp, axes=(1, 2, 3))
    Kh = np.fft.fftn(K, axes=(2, 3, 4))
    Hh = np.einsum("abzyx,bzyx->azyx", Kh, Mh)
    Hf = -np.real(np.fft.ifftn(Hh, axes=(1, 2, 3)))[:, :nz, :ny, :nx]
    Hd = oracle.field(n, h, M, full_box(n), full_box(n), table=table)
    np.testing.assert_allclose(Hf, Hd, rtol=0, atol=1e-13 * np.abs(Hd).max())
    # the tensor spectra are real (each component is even or odd per axis)
    assert np.abs(Kh.imag).max() < 1e-12 * np.abs(Kh).max()


def test_adjoint_is_the_same_operator():
    """<D a, b> = <a, D b>: the stray-field operator is self-adjoint (N
    symmetric in its components and even in the offset), the property the
    paper relies on to reuse one operator for the adjoint."""
    rng = np.random.default_rng(2)
    n, h = (7, 6, 5), (1.0, 1.3, 0.6)
    a = rng.normal(size=(3, 5, 6, 7))
    b = rng.normal(size=(3, 5, 6, 7))
    fb = full_box(n)
    Da = oracle.field(n, h, a, fb, fb)
    Db = oracle.field(n, h, b, fb, fb)
    lhs, rhs = float(np.sum(Da * b)), float(np.sum(a * Db))
    assert abs(lhs - rhs) < 1e-14 * max(abs(lhs), 1.0) * 10
