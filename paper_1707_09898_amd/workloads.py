"""Seeded synthetic workloads for the FD topology-optimization gradient.

This module only draws inputs and names geometry: grid sizes, cell sizes,
design/sensor index boxes, densities rho, magnetization directions M0 and
target fields.  It holds none of the method's arithmetic (no tensor, no
convolution, no objective), so that both the CPU oracle and the HIP path can
consume the very same arrays.

Arrays are numpy float64 in C order ``[nz][ny][nx]`` (x fastest).  FP32 runs
round them once (``astype(np.float32)``).

The paper's own workload is a synthetic geometry (a unit-cube design region
magnetized along z with a small sensing box above it, Sec. "Validation and
Benchmarks", p = 3, rho_0 = 1).  The five configurations below stand in for
it at the sizes the gradient engine is measured on.

RNG: ``numpy.random.default_rng(seed)`` (PCG64), seed = configuration number;
the batch of configuration 5 draws one stream per design from
``SeedSequence(5).spawn(64)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Objective kinds (shared names; each side implements the arithmetic itself).
J_MEAN_SQ_HZ = 1          # J = mean_s (Hz_s - t)^2
J_MEAN_SQ_HZ_GRADXY = 2   # J = mean_s (Hz_s - t)^2 + lam * mean_s (DxHz^2 + DyHz^2)
J_MEAN_SQ_H_TARGET = 3    # J = mean_s |H_s - H*_s|^2
J_NEG_HALF_HZ2 = 4        # J = -1/2 V_cell sum_s Hz_s^2   (paper's benchmark objective)
J_FIELD_GRADIENT = 5      # J = -1/2 V_cell [sum_s Hz_s^2 + beta sum_strip (D_n Hz)^2]  (field and gradient design)

Box = Tuple[int, int, int, int, int, int]  # (x0, x1, y0, y1, z0, z1), half-open


@dataclasses.dataclass
class Workload:
    """One gradient-evaluation problem on a regular cuboid grid."""

    name: str
    n: Tuple[int, int, int]            # (nx, ny, nz) cells of the FFT box
    h: Tuple[float, float, float]      # (dx, dy, dz) cell size
    design: Box                        # design region chi (index box)
    sensor: Box                        # sensor cells the objective reads
    p: int                             # penalization exponent
    rho: np.ndarray                    # [nz][ny][nx] float64
    m0: Tuple[float, float, float] = (0.0, 0.0, 1.0)   # uniform M0
    m0_field: Optional[np.ndarray] = None               # [3][nz][ny][nx] or None
    j_kind: int = J_MEAN_SQ_HZ_GRADXY
    j_target: float = 0.2
    j_lambda: float = 0.01
    h_target: Optional[np.ndarray] = None               # [3][sensor cells] (C4)
    pad: Optional[Tuple[int, int, int]] = None          # padded FFT lengths (None: rule)
    mask: Optional[np.ndarray] = None                   # [nz][ny][nx] uint8: design cells are box and mask != 0

    @property
    def cells(self) -> int:
        nx, ny, nz = self.n
        return nx * ny * nz


def box_filter3(u: np.ndarray, width: int = 3) -> np.ndarray:
    """Mean over the in-grid width^3 neighbourhood (count-normalized at borders)."""
    r = width // 2
    out = np.zeros_like(u)
    cnt = np.zeros_like(u)
    nz, ny, nx = u.shape
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                zs = slice(max(0, dz), nz + min(0, dz))
                zd = slice(max(0, -dz), nz + min(0, -dz))
                ys = slice(max(0, dy), ny + min(0, dy))
                yd = slice(max(0, -dy), ny + min(0, -dy))
                xs = slice(max(0, dx), nx + min(0, dx))
                xd = slice(max(0, -dx), nx + min(0, -dx))
                out[zd, yd, xd] += u[zs, ys, xs]
                cnt[zd, yd, xd] += 1.0
    return out / cnt


def _rescale(u: np.ndarray, lo: float, hi: float) -> np.ndarray:
    a, b = float(u.min()), float(u.max())
    return lo + (hi - lo) * (u - a) / (b - a)


def _smooth_field(rng: np.random.Generator, shape, lo, hi) -> np.ndarray:
    u = rng.random(shape)
    u = box_filter3(box_filter3(u, 9), 9)
    return _rescale(u, lo, hi)


def config1() -> Workload:
    """16^3 unit cubes, sensor = 8 cells on a line 2 cells above the top face.

    The FFT box is extended to 16x16x18 so that the sensor layer (k = 17) is
    inside it; the design region is k in [0, 16).
    """
    rng = np.random.default_rng(1)
    n = (16, 16, 18)
    rho = rng.random((n[2], n[1], n[0]))
    return Workload(name="c1_16x16x16", n=n, h=(1.0, 1.0, 1.0),
                    design=(0, 16, 0, 16, 0, 16), sensor=(8, 9, 4, 12, 17, 18),
                    p=3, rho=rho, j_kind=J_MEAN_SQ_HZ, j_target=0.1, j_lambda=0.0)


def config2() -> Workload:
    """64^3 grid, cells 1 x 1 x 0.5, box-filtered rho, sensor plane 4 cells up."""
    rng = np.random.default_rng(2)
    n = (64, 64, 64)
    rho = box_filter3(rng.random((n[2], n[1], n[0])), 3)
    return Workload(name="c2_64x64x64", n=n, h=(1.0, 1.0, 0.5),
                    design=(0, 64, 0, 64, 0, 32), sensor=(24, 40, 24, 40, 35, 36),
                    p=3, rho=rho, j_kind=J_MEAN_SQ_HZ_GRADXY, j_target=0.2, j_lambda=0.01)


def config3() -> Workload:
    """256 x 256 x 128 cubic cells (padded 512 x 512 x 256), 64 x 64 sensor plane."""
    rng = np.random.default_rng(3)
    n = (256, 256, 128)
    rho = rng.random((n[2], n[1], n[0]))
    return Workload(name="c3_256x256x128", n=n, h=(1.0, 1.0, 1.0),
                    design=(0, 256, 0, 256, 0, 124), sensor=(96, 160, 96, 160, 127, 128),
                    p=3, rho=rho, j_kind=J_MEAN_SQ_HZ_GRADXY, j_target=0.2, j_lambda=0.01)


def config4() -> Workload:
    """128 x 128 x 64, spatially varying unit M0, 32 x 32 x 4 sensor box, target H*."""
    rng = np.random.default_rng(4)
    n = (128, 128, 64)
    shape = (n[2], n[1], n[0])
    rho = rng.random(shape)
    theta = math.pi * _smooth_field(rng, shape, 0.0, 1.0)
    phi = 2.0 * math.pi * _smooth_field(rng, shape, 0.0, 1.0)
    m0 = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    sensor = (48, 80, 48, 80, 60, 64)
    sshape = (sensor[5] - sensor[4], sensor[3] - sensor[2], sensor[1] - sensor[0])
    ht = np.stack([0.05 * _smooth_field(rng, sshape, -1.0, 1.0) for _ in range(3)])
    return Workload(name="c4_128x128x64", n=n, h=(1.0, 1.0, 1.0),
                    design=(0, 128, 0, 128, 0, 56), sensor=sensor, p=3, rho=rho,
                    m0_field=m0, j_kind=J_MEAN_SQ_H_TARGET, j_target=0.0, j_lambda=0.0,
                    h_target=ht)


def config5(count: int = 64) -> List[Workload]:
    """A batch of independent designs of uneven size and cell aspect."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(5).spawn(count)):
        rng = np.random.default_rng(ss)
        nx = int(rng.integers(32, 161))
        ny = int(rng.integers(32, 161))
        nz = int(rng.integers(32, 97))
        h = tuple(float(v) for v in rng.uniform(0.5, 2.0, 3))
        p = int(rng.integers(3, 5))
        rho = box_filter3(rng.random((nz, ny, nx)), 3)
        kd = nz // 2
        ks = kd - 1 + 4
        sx, sy = nx // 4, ny // 4
        x0, y0 = (nx - sx) // 2, (ny - sy) // 2
        out.append(Workload(name=f"c5_{i:02d}_{nx}x{ny}x{nz}", n=(nx, ny, nz), h=h,
                            design=(0, nx, 0, ny, 0, kd),
                            sensor=(x0, x0 + sx, y0, y0 + sy, ks, ks + 1), p=p, rho=rho,
                            j_kind=J_MEAN_SQ_HZ_GRADXY, j_target=0.2, j_lambda=0.01))
    return out


def small_random(seed: int, n=(12, 10, 14), h=(1.0, 1.0, 1.0), design=None, sensor=None,
                 p: int = 3, j_kind: int = J_MEAN_SQ_HZ_GRADXY, varying_m0: bool = False,
                 m0=(0.0, 0.0, 1.0)) -> Workload:
    """Small seeded problems for parity tests (ragged sizes, several tiles)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    shape = (nz, ny, nx)
    rho = rng.random(shape)
    if design is None:
        design = (0, nx, 0, ny, 0, max(1, nz - 4))
    if sensor is None:
        sx, sy = max(1, nx // 3), max(1, ny // 3)
        x0, y0 = (nx - sx) // 2, (ny - sy) // 2
        sensor = (x0, x0 + sx, y0, y0 + sy, nz - 1, nz)
    m0_field = None
    ht = None
    if varying_m0:
        v = rng.normal(size=(3,) + shape)
        m0_field = v / np.linalg.norm(v, axis=0, keepdims=True)
    if j_kind == J_MEAN_SQ_H_TARGET:
        sshape = (sensor[5] - sensor[4], sensor[3] - sensor[2], sensor[1] - sensor[0])
        ht = 0.05 * rng.uniform(-1.0, 1.0, (3,) + sshape)
    return Workload(name=f"small_{seed}", n=n, h=h, design=design, sensor=sensor, p=p,
                    rho=rho, m0=m0, m0_field=m0_field, j_kind=j_kind, j_target=0.2,
                    j_lambda={J_MEAN_SQ_HZ_GRADXY: 0.01, J_FIELD_GRADIENT: 0.5}.get(j_kind, 0.0),
                    h_target=ht)


def random_mask(seed: int, n, fraction: float = 0.7) -> np.ndarray:
    """A seeded uint8 design mask [nz][ny][nx]: each cell kept with probability `fraction`."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return (rng.random((nz, ny, nx)) < fraction).astype(np.uint8)


def by_name(name: str):
    return {"c1": config1, "c2": config2, "c3": config3, "c4": config4}[name]()
