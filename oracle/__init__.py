"""CPU oracle for the FD topology-optimization gradient (Abert et al. 2017).

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct FP64 definitions
that the HIP path is checked against.  Only ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product path
never does, and this package imports nothing of the product (only the seeded
input generators, which hold no arithmetic of the method).

Where each step comes from (paper sections and equations):

* ``magnetization``  M = chi rho^p M0 (Sec. "Methodology", the penalized
  magnetization M(rho) = rho^p M0; chi is the design region's characteristic
  function, as in the benchmark section: an index box, optionally intersected
  with a cell mask, ``design_chi``).
* ``newell_table``   the discrete demagnetization tensor, eq. (demag_tensor),
  in quad precision (C, ``oracle.c``).
* ``field``          the discrete convolution, eq. (convolution), as a direct
  sum (C).  Field H = -N (*) M with the positive Newell tensor N.
* ``objective``      J(H) and the exact discrete dJ/dH of the objective kinds
  (eq. (objective_function) in its general form; the configurations fix J).
* ``gradient``       chain rule for the discrete problem, the adjoint form of
  eqs. (dj_drho), (adjoint1), (adjoint2): dJ/drho_j = chi_j p rho_j^(p-1)
  M0_j . D(dJ/dH)_j + dJ/drho_j(explicit), where D is the same stray-field
  operator as the forward one (N symmetric and even).  The paper prints this
  with a leading minus sign; differentiating the discrete J directly gives a
  plus sign, and the finite-difference tests pin the plus sign.
* ``project_step``   one step of the bound-constrained update that keeps
  0 <= rho <= 1 (Sec. Methodology relaxes rho to [0, 1]; Sec. Discretization
  minimizes with a quasi-Newton method that handles that bound).  The measured
  loop uses the simplest such method, a projected gradient step normalized by
  the largest gradient magnitude on the design cells; its definition is
  written out here.

Parity pins are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

XX, YY, ZZ, XY, XZ, YZ = range(6)
J_MEAN_SQ_HZ, J_MEAN_SQ_HZ_GRADXY, J_MEAN_SQ_H_TARGET, J_NEG_HALF_HZ2, J_FIELD_GRADIENT = 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, libquadmath)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", _SRC,
               "-lquadmath", "-lm", "-o", _LIB_PATH]
        subprocess.check_call(cmd)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_newell_table.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [ctypes.c_int, dp]
        L.oracle_newell_table.restype = ctypes.c_int
        L.oracle_field.argtypes = ([ctypes.c_int] * 3 + [dp] + [ctypes.c_int] * 3 +
                                   [dp, ctypes.c_int, ip, ctypes.c_int, ip, dp])
        L.oracle_field.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def newell_table(m: Sequence[int], h: Sequence[float], comps: Sequence[int] = range(6)) -> np.ndarray:
    """Tensor N_c(k) for 0 <= k_a < m_a, shape [6][mz][my][mx] (NaN where not computed)."""
    mx, my, mz = (int(v) for v in m)
    out = np.full((6, mz, my, mx), np.nan)
    mask = 0
    for c in comps:
        mask |= 1 << int(c)
    rc = lib().oracle_newell_table(mx, my, mz, float(h[0]), float(h[1]), float(h[2]), mask, _dptr(out))
    if rc != 0:
        raise RuntimeError("oracle_newell_table failed")
    return out


def tensor_at(table: np.ndarray, k: Sequence[int]) -> np.ndarray:
    """Full symmetric 3x3 tensor at a signed offset k = (kx, ky, kz), by parity."""
    kx, ky, kz = (int(v) for v in k)
    e = table[:, abs(kz), abs(ky), abs(kx)]
    sx = -1.0 if kx < 0 else 1.0
    sy = -1.0 if ky < 0 else 1.0
    sz = -1.0 if kz < 0 else 1.0
    return np.array([[e[XX], sx * sy * e[XY], sx * sz * e[XZ]],
                     [sx * sy * e[XY], e[YY], sy * sz * e[YZ]],
                     [sx * sz * e[XZ], sy * sz * e[YZ], e[ZZ]]])


def _components_needed(src_mask: int, tgt_mask: int) -> list:
    out = set()
    for a in range(3):
        for b in range(3):
            if (tgt_mask >> a) & 1 and (src_mask >> b) & 1:
                if a == b:
                    out.add(a)
                else:
                    lo, hi = min(a, b), max(a, b)
                    out.add({(0, 1): XY, (0, 2): XZ, (1, 2): YZ}[(lo, hi)])
    return sorted(out)


def table_extent(sbox, tbox) -> Tuple[int, int, int]:
    """Smallest offset range [0, m) per axis that covers every target - source."""
    m = []
    for a in range(3):
        s0, s1 = sbox[2 * a], sbox[2 * a + 1]
        t0, t1 = tbox[2 * a], tbox[2 * a + 1]
        m.append(max(t1 - 1 - s0, s1 - 1 - t0, 0) + 1)
    return tuple(m)


def field(n, h, M: np.ndarray, sbox, tbox, src_mask: int = 7, tgt_mask: int = 7,
          table: Optional[np.ndarray] = None) -> np.ndarray:
    """Direct-sum stray field H = -N (*) M on the target box (zero elsewhere).

    M: [3][nz][ny][nx] float64 (source), result [3][nz][ny][nx].
    """
    nx, ny, nz = n
    M = np.ascontiguousarray(M, dtype=np.float64)
    assert M.shape == (3, nz, ny, nx)
    m = table_extent(sbox, tbox)
    if table is None:
        table = newell_table(m, h, _components_needed(src_mask, tgt_mask))
    else:
        assert all(table.shape[3 - a] >= m[a] for a in range(3))
    table = np.ascontiguousarray(table)
    tz, ty, tx = table.shape[1:]
    H = np.zeros((3, nz, ny, nx))
    sb = np.array(sbox, dtype=np.int32)
    tb = np.array(tbox, dtype=np.int32)
    rc = lib().oracle_field(nx, ny, nz, _dptr(table), tx, ty, tz, _dptr(M), int(src_mask),
                            _iptr(sb), int(tgt_mask), _iptr(tb), _dptr(H))
    if rc != 0:
        raise RuntimeError("oracle_field failed")
    return H


def box_mask(n, box) -> np.ndarray:
    """Characteristic function of an index box, [nz][ny][nx]."""
    nx, ny, nz = n
    chi = np.zeros((nz, ny, nx))
    x0, x1, y0, y1, z0, z1 = box
    chi[z0:z1, y0:y1, x0:x1] = 1.0
    return chi


def design_chi(w) -> np.ndarray:
    """chi of the design region: 1 on the cells of the design box whose mask
    entry (if the workload has a mask) is nonzero, 0 elsewhere."""
    chi = box_mask(w.n, w.design)
    if getattr(w, "mask", None) is not None:
        chi = chi * (np.asarray(w.mask) != 0)
    return chi


def ipow(x: np.ndarray, p: int) -> np.ndarray:
    """x^p for integer p >= 0 by repeated multiplication."""
    r = np.ones_like(x)
    for _ in range(p):
        r = r * x
    return r


def m0_array(w) -> np.ndarray:
    nx, ny, nz = w.n
    if w.m0_field is not None:
        return np.asarray(w.m0_field, dtype=np.float64)
    return np.broadcast_to(np.asarray(w.m0, dtype=np.float64)[:, None, None, None], (3, nz, ny, nx)).copy()


def magnetization(w, rho: Optional[np.ndarray] = None) -> np.ndarray:
    """M = chi rho^p M0 (Sec. Methodology), [3][nz][ny][nx]."""
    rho = w.rho if rho is None else rho
    chi = design_chi(w)
    return (chi * ipow(rho, w.p))[None] * m0_array(w)


def m0_mask(w) -> int:
    if w.m0_field is not None:
        return 7
    return sum(1 << a for a in range(3) if w.m0[a] != 0.0)


def objective_box(w):
    """Cells J reads: the sensor, widened by one cell in x and y for the
    gradient term (kind 2), or by the strip and its outer neighbours, two
    cells, on the -x, +x and -y sides (kind 5)."""
    x0, x1, y0, y1, z0, z1 = w.sensor
    nx, ny, _ = w.n
    if w.j_kind == J_MEAN_SQ_HZ_GRADXY:
        if x0 < 1 or y0 < 1 or x1 > nx - 1 or y1 > ny - 1:
            raise ValueError("sensor must have in-grid x/y neighbours for the gradient term")
        return (x0 - 1, x1 + 1, y0 - 1, y1 + 1, z0, z1)
    if w.j_kind == J_FIELD_GRADIENT:
        if x0 < 2 or y0 < 2 or x1 > nx - 2:
            raise ValueError("the gradient strip and its outer neighbours must be in the grid")
        return (x0 - 2, x1 + 2, y0 - 2, y1, z0, z1)
    return tuple(w.sensor)


def gradient_strip(w):
    """The cells of the gradient region of kind 5 with their outward normal:
    a one-cell strip outside the field region on its -x, +x and -y sides, as
    (z, y, x, axis, sign) with axis 0 = x, 1 = y."""
    x0, x1, y0, y1, z0, z1 = w.sensor
    out = []
    for z in range(z0, z1):
        for y in range(y0, y1):
            out.append((z, y, x0 - 1, 0, -1))
            out.append((z, y, x1, 0, +1))
        for x in range(x0, x1):
            out.append((z, y0 - 1, x, 1, -1))
    return out


def objective_mask(w) -> int:
    return 7 if w.j_kind == J_MEAN_SQ_H_TARGET else 4


def objective(w, H: np.ndarray) -> Tuple[float, np.ndarray]:
    """J(H) and g = dJ/dH (exact discrete derivative), g shaped like H ([3][nz][ny][nx]).

    H must hold the field on objective_box(w).
    """
    x0, x1, y0, y1, z0, z1 = w.sensor
    S = (x1 - x0) * (y1 - y0) * (z1 - z0)
    g = np.zeros_like(H)
    hz = H[2]
    if w.j_kind == J_MEAN_SQ_HZ:
        d = hz[z0:z1, y0:y1, x0:x1] - w.j_target
        J = float(np.sum(d * d)) / S
        g[2, z0:z1, y0:y1, x0:x1] = 2.0 * d / S
    elif w.j_kind == J_MEAN_SQ_HZ_GRADXY:
        dx, dy, _ = w.h
        d = hz[z0:z1, y0:y1, x0:x1] - w.j_target
        # central differences over in-grid neighbours
        Dx = (hz[z0:z1, y0:y1, x0 + 1:x1 + 1] - hz[z0:z1, y0:y1, x0 - 1:x1 - 1]) / (2.0 * dx)
        Dy = (hz[z0:z1, y0 + 1:y1 + 1, x0:x1] - hz[z0:z1, y0 - 1:y1 - 1, x0:x1]) / (2.0 * dy)
        lam = w.j_lambda
        J = float(np.sum(d * d)) / S + lam * float(np.sum(Dx * Dx) + np.sum(Dy * Dy)) / S
        g[2, z0:z1, y0:y1, x0:x1] += 2.0 * d / S
        # transpose of the central differences, scattered onto the neighbours
        cx = 2.0 * lam / S * Dx / (2.0 * dx)
        cy = 2.0 * lam / S * Dy / (2.0 * dy)
        g[2, z0:z1, y0:y1, x0 + 1:x1 + 1] += cx
        g[2, z0:z1, y0:y1, x0 - 1:x1 - 1] -= cx
        g[2, z0:z1, y0 + 1:y1 + 1, x0:x1] += cy
        g[2, z0:z1, y0 - 1:y1 - 1, x0:x1] -= cy
    elif w.j_kind == J_MEAN_SQ_H_TARGET:
        d = H[:, z0:z1, y0:y1, x0:x1] - w.h_target
        J = float(np.sum(d * d)) / S
        g[:, z0:z1, y0:y1, x0:x1] = 2.0 * d / S
    elif w.j_kind == J_NEG_HALF_HZ2:
        V = w.h[0] * w.h[1] * w.h[2]
        v = hz[z0:z1, y0:y1, x0:x1]
        J = -0.5 * V * float(np.sum(v * v))
        g[2, z0:z1, y0:y1, x0:x1] = -V * v
    elif w.j_kind == J_FIELD_GRADIENT:
        # J = -1/2 V [sum_field Hz^2 + beta sum_strip (D_n Hz)^2], D_n the forward
        # difference along the strip cell's outward normal n: (Hz(s + n) - Hz(s)) / h
        V = w.h[0] * w.h[1] * w.h[2]
        beta = w.j_lambda
        v = hz[z0:z1, y0:y1, x0:x1]
        total = float(np.sum(v * v))
        g[2, z0:z1, y0:y1, x0:x1] = -V * v
        for (z, y, x, axis, sgn) in gradient_strip(w):
            hstep = w.h[axis]
            zn, yn, xn = (z, y, x + sgn) if axis == 0 else (z, y + sgn, x)
            D = (hz[zn, yn, xn] - hz[z, y, x]) / hstep
            total += beta * D * D
            c = -V * beta * D / hstep
            g[2, zn, yn, xn] += c
            g[2, z, y, x] -= c
        J = -0.5 * V * total
    else:
        raise ValueError(f"unknown objective kind {w.j_kind}")
    return J, g


def forward_field(w, rho: Optional[np.ndarray] = None, tbox=None, tgt_mask: Optional[int] = None,
                  table: Optional[np.ndarray] = None) -> np.ndarray:
    """H on a target box (default: the cells the objective reads)."""
    tbox = objective_box(w) if tbox is None else tbox
    tgt_mask = objective_mask(w) if tgt_mask is None else tgt_mask
    M = magnetization(w, rho)
    return field(w.n, w.h, M, w.design, tbox, m0_mask(w), tgt_mask, table)


def adjoint_field(w, g: np.ndarray, table: Optional[np.ndarray] = None) -> np.ndarray:
    """A = D(g) on the design box: the same stray-field operator applied to dJ/dH."""
    return field(w.n, w.h, g, objective_box(w), w.design, objective_mask(w), m0_mask(w), table)


def gradient_from_adjoint(w, A: np.ndarray, rho: Optional[np.ndarray] = None) -> np.ndarray:
    """dJ/drho = chi p rho^(p-1) M0 . A  (explicit dJ/drho is zero for these objectives)."""
    rho = w.rho if rho is None else rho
    chi = design_chi(w)
    return chi * w.p * ipow(rho, w.p - 1) * np.sum(m0_array(w) * A, axis=0)


def table_for(w) -> np.ndarray:
    """One tensor table that covers both the forward and the adjoint offsets."""
    tb = objective_box(w)
    m = table_extent(w.design, tb)
    comps = _components_needed(m0_mask(w), objective_mask(w))
    return newell_table(m, w.h, comps)


def objective_and_grad(w, rho: Optional[np.ndarray] = None, table: Optional[np.ndarray] = None):
    """(J, dJ/drho [nz][ny][nx], H on the objective box) for one density field."""
    table = table_for(w) if table is None else table
    H = forward_field(w, rho, table=table)
    J, g = objective(w, H)
    A = adjoint_field(w, g, table=table)
    return J, gradient_from_adjoint(w, A, rho), H


def project_step(w, rho: np.ndarray, grad: np.ndarray, alpha: float) -> np.ndarray:
    """One projected-gradient update of the density (a new array):

        rho_j <- min(1, max(0, rho_j - alpha * grad_j / G)),  G = max over chi of |grad|,

    on the design cells j (chi_j = 1); every other cell keeps its value, and
    G = 0 leaves rho unchanged.  FP64."""
    chi = design_chi(w) != 0
    rho = np.asarray(rho, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    G = float(np.abs(grad[chi]).max()) if chi.any() else 0.0
    if G == 0.0:
        return rho.copy()
    moved = np.minimum(1.0, np.maximum(0.0, rho - alpha * grad / G))
    return np.where(chi, moved, rho)
