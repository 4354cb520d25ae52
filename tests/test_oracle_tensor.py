"""Pins of the oracle's demagnetization tensor (eq. (demag_tensor)) against
things other than its own formula: closed forms for a single prism, the
trace identity of the Laplacian, the block (aggregation) identity of the
defining sixfold integral, an independent numerical quadrature of that
integral, and the dipole limit."""
import itertools
import math

import mpmath
import numpy as np
import pytest

import oracle


def aharoni_nz(a: float, b: float, c: float) -> float:
    """Demagnetizing factor along z of a 2a x 2b x 2c prism (Aharoni, J. Appl.
    Phys. 83, 3432 (1998), eq. (1)), evaluated with mpmath at 40 digits."""
    mpmath.mp.dps = 40
    a, b, c = mpmath.mpf(a), mpmath.mpf(b), mpmath.mpf(c)
    abc = mpmath.sqrt(a * a + b * b + c * c)
    ab = mpmath.sqrt(a * a + b * b)
    bc = mpmath.sqrt(b * b + c * c)
    ac = mpmath.sqrt(a * a + c * c)
    ln = mpmath.log
    r = ((b * b - c * c) / (2 * b * c) * ln((abc - a) / (abc + a))
         + (a * a - c * c) / (2 * a * c) * ln((abc - b) / (abc + b))
         + b / (2 * c) * ln((ab + a) / (ab - a))
         + a / (2 * c) * ln((ab + b) / (ab - b))
         + c / (2 * a) * ln((bc - b) / (bc + b))
         + c / (2 * b) * ln((ac - a) / (ac + a))
         + 2 * mpmath.atan(a * b / (c * abc))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * abc
         + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return float(r / mpmath.pi)


def self_term(h):
    return oracle.newell_table((1, 1, 1), h)[:, 0, 0, 0]


@pytest.mark.parametrize("edge", [1.0, 2.5, 0.3])
def test_cube_self_term_is_one_third(edge):
    t = self_term((edge, edge, edge))
    np.testing.assert_allclose(t[:3], 1.0 / 3.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(t[3:], 0.0, atol=1e-15)


@pytest.mark.parametrize("h", [(1.0, 1.0, 0.5), (0.7, 1.3, 2.0), (2.0, 0.5, 1.1), (1.0, 1.0, 10.0)])
def test_self_term_matches_aharoni_prism(h):
    t = self_term(h)
    a, b, c = (v / 2 for v in h)
    assert abs(t[2] - aharoni_nz(a, b, c)) < 1e-14
    assert abs(t[0] - aharoni_nz(b, c, a)) < 1e-14
    assert abs(t[1] - aharoni_nz(c, a, b)) < 1e-14
    assert abs(t[0] + t[1] + t[2] - 1.0) < 1e-14


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (1.0, 1.0, 0.5), (0.7, 1.3, 2.0)])
def test_trace_vanishes_off_origin(h):
    # Laplacian of 1/r vanishes away from the origin; cell averaging keeps it
    t = oracle.newell_table((7, 6, 5), h)
    tr = t[0] + t[1] + t[2]
    tr[0, 0, 0] -= 1.0
    scale = np.abs(t[:3]).max()
    assert np.abs(tr).max() < 1e-14 * scale


def block_mean(table, B, K):
    """(1/#cells) sum_{i in block at K, j in block at 0} N_small(i - j), all 6 comps."""
    Bx, By, Bz = B
    acc = np.zeros((3, 3))
    cells = list(itertools.product(range(Bx), range(By), range(Bz)))
    for (ix, iy, iz) in cells:
        for (jx, jy, jz) in cells:
            k = (K[0] * Bx + ix - jx, K[1] * By + iy - jy, K[2] * Bz + iz - jz)
            acc += oracle.tensor_at(table, k)
    return acc / len(cells)


@pytest.mark.parametrize("B,h,K", [((2, 1, 1), (1.0, 1.0, 1.0), (0, 0, 0)),
                                   ((2, 2, 1), (1.0, 1.0, 0.5), (1, 0, 2)),
                                   ((3, 2, 2), (0.7, 1.3, 2.0), (1, -1, 1)),
                                   ((2, 3, 2), (1.0, 1.0, 1.0), (-2, 1, 3))])
def test_block_identity(B, h, K):
    """The tensor of aggregated cells equals the mean over the fine cell pairs.

    Follows from the sixfold integral of eq. (demag_tensor): integrating over a
    union of cells is the sum of the integrals over its cells.  Pins the
    stencil, its weights and the signs of the off-diagonal components."""
    m = tuple(abs(K[a]) * B[a] + B[a] for a in range(3))
    fine = oracle.newell_table(m, h)
    big_h = tuple(B[a] * h[a] for a in range(3))
    coarse = oracle.newell_table(tuple(abs(K[a]) + 1 for a in range(3)), big_h)
    want = oracle.tensor_at(coarse, K)
    got = block_mean(fine, B, K)
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-14 * max(scale, 1e-3))
    if K == (0, 0, 0):
        assert abs(np.trace(got) - 1.0) < 1e-14


def quadrature_tensor(r, h, npts=16):
    """N_ab(r) = -(1/4piV) int Lambda(s) d_a d_b (1/|r+s|) ds, Lambda the cell
    autocorrelation prod_c (h_c - |s_c|); Gauss-Legendre on the 8 kink-free
    sub-boxes.  Valid away from the origin (the integrand is then smooth)."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    nodes, weights = [], []
    for c in range(3):
        # [-h, 0] and [0, h]
        s = np.concatenate([(xg - 1) * h[c] / 2, (xg + 1) * h[c] / 2])
        w = np.concatenate([wg, wg]) * h[c] / 2 * (h[c] - np.abs(s))
        nodes.append(s)
        weights.append(w)
    sx, sy, sz = np.meshgrid(*nodes, indexing="ij")
    W = np.einsum("i,j,k->ijk", *weights)
    q = np.stack([r[0] + sx, r[1] + sy, r[2] + sz])
    q2 = np.sum(q * q, axis=0)
    q5 = q2 ** 2.5
    V = h[0] * h[1] * h[2]
    out = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            kern = (3 * q[a] * q[b] - (q2 if a == b else 0.0)) / q5
            out[a, b] = -np.sum(W * kern) / (4 * math.pi * V)
    return out


@pytest.mark.parametrize("k,h", [((3, 1, 0), (1.0, 1.0, 1.0)), ((4, -2, 3), (1.0, 1.0, 0.5)),
                                 ((-3, 5, 2), (0.7, 1.3, 2.0)), ((6, 3, -4), (1.0, 1.0, 1.0))])
def test_independent_quadrature(k, h):
    m = tuple(abs(v) + 1 for v in k)
    t = oracle.newell_table(m, h)
    got = oracle.tensor_at(t, k)
    r = tuple(k[a] * h[a] for a in range(3))
    want = quadrature_tensor(r, h, npts=24)
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * scale)


def dipole(r, V):
    r = np.asarray(r, dtype=float)
    rr = float(r @ r)
    return V / (4 * math.pi) * (np.eye(3) * rr - 3 * np.outer(r, r)) / rr ** 2.5


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.7, 1.3, 2.0)])
def test_dipole_limit(h):
    """Far away the cell pair interacts like two point dipoles; the deviation
    falls like (cell/r)^2, so doubling the distance cuts it about fourfold."""
    k1 = (6, 3, 2)
    k2 = (12, 6, 4)
    t = oracle.newell_table((13, 7, 5), h)
    V = h[0] * h[1] * h[2]
    devs = []
    for k in (k1, k2):
        r = [k[a] * h[a] for a in range(3)]
        d = dipole(r, V)
        devs.append(np.abs(oracle.tensor_at(t, k) - d).max() / np.abs(d).max())
    assert devs[0] < 0.1
    assert devs[1] < devs[0] / 3.0


def test_parity_by_direct_quadrature():
    """Odd components flip sign with the offset, diagonal ones do not; checked
    against the quadrature at all eight sign combinations of one offset."""
    h = (1.0, 1.0, 0.5)
    t = oracle.newell_table((4, 4, 5), h)
    for sx, sy, sz in itertools.product((-1, 1), repeat=3):
        k = (3 * sx, 2 * sy, 4 * sz)
        r = tuple(k[a] * h[a] for a in range(3))
        want = quadrature_tensor(r, h, npts=20)
        np.testing.assert_allclose(oracle.tensor_at(t, k), want, rtol=0,
                                   atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("k,h", [((150, 90, 60), (1.0, 1.0, 1.0)), ((255, 160, 127), (1.0, 1.0, 1.0)),
                                 ((40, 33, 25), (0.7, 1.3, 2.0))])
def test_far_offsets_are_accurate(k, h):
    """At large offsets the second difference cancels O(r^6) relative; double
    precision would lose 1e-5..1e-1 here.  The quadrature of the defining
    integral (smooth integrand this far out) pins the quad-precision lattice
    to 1e-12 relative."""
    big = max(k) > 100
    comps = [2, 4] if big else list(range(6))   # zz and xz suffice for the largest offset
    t = oracle.newell_table(tuple(v + 1 for v in k), h, comps)
    got = oracle.tensor_at(np.nan_to_num(t), k)
    r = tuple(k[a] * h[a] for a in range(3))
    want = quadrature_tensor(r, h, npts=8)
    pairs = [(2, 2), (0, 2)] if big else [(a, b) for a in range(3) for b in range(3)]
    for a, b in pairs:
        assert abs(got[a, b] - want[a, b]) < 1e-12 * np.abs(want).max(), (a, b)
