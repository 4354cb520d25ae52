"""Python binding of the C ABI in include/tof.h (argument marshalling only).

Every step of the gradient evaluation runs in the HIP kernels of libtof.so;
PyTorch only provides device memory and the current stream.  Importing this
module does not need a GPU; creating an Engine does, and fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtof.so")

TOF_F32, TOF_F64 = 1, 2
J_MEAN_SQ_HZ, J_MEAN_SQ_HZ_GRADXY, J_MEAN_SQ_H_TARGET, J_NEG_HALF_HZ2, J_FIELD_GRADIENT = 1, 2, 3, 4, 5

STATUS = {0: "TOF_OK", -1: "TOF_ERR_INVALID", -2: "TOF_ERR_UNSUPPORTED", -3: "TOF_ERR_OOM",
          -4: "TOF_ERR_HIP", -5: "TOF_ERR_NUMERIC", -6: "TOF_ERR_STATE"}

EXPORTS = ["tof_create", "tof_destroy", "tof_set_design", "tof_set_objective", "tof_field",
           "tof_objective_and_grad", "tof_adjoint", "tof_project_step", "tof_project_step_static", "tof_tensor",
           "tof_tensor_full",
           "tof_padded_lengths", "tof_workspace_bytes", "tof_ctx_bytes", "tof_last_error", "tof_dd_newell_host",
           "tof_profile_enable", "tof_profile_read", "tof_profile_kernel", "tof_profile_burst",
           "tof_profile_burst_read", "tof_set_option", "tof_batch_create", "tof_batch_run", "tof_batch_launches", "tof_batch_destroy"]

OPT_ZSUM, OPT_FUSE_YZ, OPT_FUSE_OBJECTIVE = 1, 2, 3
OPT_X_TILE, OPT_GATHER_GROUPS, OPT_SCATTER_GROUPS = 4, 5, 6
X_TILE_AUTO, X_TILE_FULL, X_TILE_PAIR = 0, 1, 2
GRID_SELFTEST_PERTURB = 1

PROFILE_SLOTS = 12
PROFILE_NAMES = ["fwd_x", "fwd_y", "fwd_z_product", "fwd_inv_y", "fwd_inv_x_field", "objective",
                 "adj_x", "adj_y", "adj_z_product", "adj_inv_y", "adj_inv_x_grad", "j_final"]


class TofError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("Lz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("validate", ctypes.c_int32), ("flags", ctypes.c_int32)]


class BoxC(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("x0", "x1", "y0", "y1", "z0", "z1")]


class Objective(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("sensor", BoxC), ("target", ctypes.c_double),
                ("lambda_grad", ctypes.c_double), ("h_target_host", ctypes.POINTER(ctypes.c_double)),
                ("h_target_dev", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libtof.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.tof_create.argtypes = [ctypes.POINTER(Grid), vp, ctypes.POINTER(vp)]
        L.tof_destroy.argtypes = [vp]
        L.tof_destroy.restype = None
        L.tof_set_design.argtypes = [vp, ctypes.POINTER(BoxC), vp, ctypes.POINTER(dbl), vp, i32]
        L.tof_set_objective.argtypes = [vp, ctypes.POINTER(Objective)]
        L.tof_field.argtypes = [vp, vp, vp, i32, vp]
        L.tof_objective_and_grad.argtypes = [vp, vp, vp, vp, vp]
        L.tof_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.tof_project_step.argtypes = [vp, vp, vp, dbl, vp]
        L.tof_project_step_static.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(BoxC), vp, vp, vp, dbl, vp]
        L.tof_tensor.argtypes = [vp, vp, vp]
        L.tof_tensor_full.argtypes = [vp, vp, vp]
        L.tof_padded_lengths.argtypes = [vp, ctypes.POINTER(i32)]
        L.tof_workspace_bytes.argtypes = [ctypes.POINTER(Grid)]
        L.tof_workspace_bytes.restype = ctypes.c_size_t
        L.tof_ctx_bytes.argtypes = [vp]
        L.tof_ctx_bytes.restype = ctypes.c_size_t
        L.tof_last_error.argtypes = [vp]
        L.tof_last_error.restype = ctypes.c_char_p
        L.tof_dd_newell_host.argtypes = [i32, i32, i32, i32, dbl, dbl, dbl]
        L.tof_dd_newell_host.restype = dbl
        L.tof_profile_enable.argtypes = [vp, i32]
        L.tof_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(dbl)]
        L.tof_profile_kernel.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
        L.tof_profile_kernel.restype = ctypes.c_char_p
        L.tof_profile_burst.argtypes = [vp, ctypes.c_uint32, i32]
        L.tof_profile_burst_read.argtypes = [vp, ctypes.POINTER(dbl)]
        L.tof_set_option.argtypes = [vp, i32, i32]
        L.tof_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       i32, ctypes.POINTER(vp)]
        L.tof_batch_run.argtypes = [vp, vp]
        L.tof_batch_launches.argtypes = [vp]
        L.tof_batch_launches.restype = i32
        L.tof_batch_destroy.argtypes = [vp]
        L.tof_batch_destroy.restype = None
        for name in ("tof_create", "tof_set_design", "tof_set_objective", "tof_field",
                     "tof_objective_and_grad", "tof_adjoint", "tof_project_step", "tof_project_step_static",
                     "tof_tensor", "tof_tensor_full", "tof_padded_lengths", "tof_profile_enable", "tof_profile_read",
                     "tof_profile_burst", "tof_profile_burst_read", "tof_set_option", "tof_batch_create", "tof_batch_run"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _box(b) -> BoxC:
    return BoxC(*(int(v) for v in b))


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Engine:
    """One context: a grid, its FFT plans, workspaces and tensor spectra."""

    def __init__(self, n: Sequence[int], h: Sequence[float], dtype: str = "f32",
                 L: Optional[Sequence[int]] = None, stream=None, validate: bool = False, flags: int = 0):
        import torch
        self.torch = torch
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.dtype = {"f32": torch.float32, "f64": torch.float64}[dtype]
        g = make_grid(self.n, self.h, dtype, L, validate, flags)
        self._ctx = ctypes.c_void_p()
        self._keep = {}
        st = lib().tof_create(ctypes.byref(g), _stream_ptr(stream), ctypes.byref(self._ctx))
        if st != 0:
            raise TofError(st, lib().tof_last_error(None).decode())

    # -- helpers --
    def _check(self, st: int):
        if st != 0:
            raise TofError(st, lib().tof_last_error(self._ctx).decode())

    def _arr(self, t, shape, dtype=None):
        dtype = self.dtype if dtype is None else dtype
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected a contiguous {dtype} cuda tensor of shape {tuple(shape)}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        return ctypes.c_void_p(t.data_ptr())

    @property
    def shape(self) -> Tuple[int, int, int]:
        nx, ny, nz = self.n
        return (nz, ny, nx)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().tof_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup --
    def set_design(self, design=None, m0=(0.0, 0.0, 1.0), m0_field=None, p: int = 3, mask=None):
        bx = ctypes.byref(_box(design)) if design is not None else None
        m0a = (ctypes.c_double * 3)(*[float(v) for v in m0])
        mf = self._arr(m0_field, (3,) + self.shape) if m0_field is not None else None
        mk = self._arr(mask, self.shape, self.torch.uint8) if mask is not None else None
        self._keep["m0_field"] = m0_field
        self._keep["mask"] = mask
        self._check(lib().tof_set_design(self._ctx, bx, mk, m0a, mf, int(p)))

    def set_objective(self, kind: int, sensor, target: float = 0.0, lam: float = 0.0, h_target=None):
        """h_target: H* for kind 3 as a host array, or a float64 cuda tensor
        (passed as the device pointer), [3][sensor cells]."""
        import numpy as np
        ptr, dptr = None, None
        if h_target is not None:
            if isinstance(h_target, self.torch.Tensor) and h_target.device.type == "cuda":
                x0, x1, y0, y1, z0, z1 = (int(v) for v in sensor)
                dptr = self._arr(h_target, (3, z1 - z0, y1 - y0, x1 - x0), self.torch.float64)
            else:
                ht = np.ascontiguousarray(h_target, dtype=np.float64)
                self._keep["h_target"] = ht
                ptr = ht.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        obj = Objective(int(kind), _box(sensor), float(target), float(lam), ptr, dptr)
        self._check(lib().tof_set_objective(self._ctx, ctypes.byref(obj)))

    # -- hot calls --
    def field(self, rho, comps: int = 7, out=None, stream=None):
        c = bin(comps).count("1")
        if out is None:
            out = self.torch.empty((c,) + self.shape, dtype=self.dtype, device=rho.device)
        self._check(lib().tof_field(self._ctx, self._arr(rho, self.shape), self._arr(out, (c,) + self.shape),
                                    int(comps), _stream_ptr(stream)))
        return out

    def objective_and_grad(self, rho, grad=None, J=None, stream=None):
        if grad is None:
            grad = self.torch.empty(self.shape, dtype=self.dtype, device=rho.device)
        if J is None:
            J = self.torch.empty((1,), dtype=self.torch.float64, device=rho.device)
        self._check(lib().tof_objective_and_grad(self._ctx, self._arr(rho, self.shape),
                                                 self._arr(J, (1,), self.torch.float64),
                                                 self._arr(grad, self.shape), _stream_ptr(stream)))
        return J, grad

    def adjoint(self, rho, gH, grad=None, stream=None):
        if grad is None:
            grad = self.torch.empty(self.shape, dtype=self.dtype, device=rho.device)
        self._check(lib().tof_adjoint(self._ctx, self._arr(rho, self.shape), self._arr(gH, (3,) + self.shape),
                                      self._arr(grad, self.shape), _stream_ptr(stream)))
        return grad

    def project_step(self, rho, grad, alpha: float, stream=None):
        self._check(lib().tof_project_step(self._ctx, self._arr(rho, self.shape), self._arr(grad, self.shape),
                                           float(alpha), _stream_ptr(stream)))
        return rho

    # -- checks / introspection --
    def tensor(self, stream=None):
        N = self.torch.empty((6,) + self.shape, dtype=self.torch.float64, device="cuda")
        self._check(lib().tof_tensor(self._ctx, ctypes.c_void_p(N.data_ptr()), _stream_ptr(stream)))
        return N

    def tensor_full(self, stream=None):
        """The tensor at every signed offset, [6][2nz-1][2ny-1][2nx-1] (tof_tensor_full)."""
        nx, ny, nz = self.n
        N = self.torch.empty((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1), dtype=self.torch.float64, device="cuda")
        self._check(lib().tof_tensor_full(self._ctx, ctypes.c_void_p(N.data_ptr()), _stream_ptr(stream)))
        return N

    def profile(self, enable: bool = True):
        self._check(lib().tof_profile_enable(self._ctx, 1 if enable else 0))

    def profile_read(self):
        """Per slot: (name, total ms, launches, algorithmic bytes per launch)."""
        ms = (ctypes.c_double * PROFILE_SLOTS)()
        cnt = (ctypes.c_int64 * PROFILE_SLOTS)()
        by = (ctypes.c_double * PROFILE_SLOTS)()
        self._check(lib().tof_profile_read(self._ctx, ms, cnt, by))
        return [(PROFILE_NAMES[i], ms[i], cnt[i], by[i]) for i in range(PROFILE_SLOTS)]

    def profile_burst(self, slots, repeats: int):
        """Arm a burst of `repeats` extra back-to-back launches for every slot
        in `slots` (indices) at the next call (tof_profile_burst)."""
        mask = 0
        for i in slots:
            mask |= 1 << int(i)
        self._check(lib().tof_profile_burst(self._ctx, mask, int(repeats)))

    def profile_burst_read(self):
        """Per slot: mean ms per launch of its last burst, 0.0 where none ran."""
        ms = (ctypes.c_double * PROFILE_SLOTS)()
        self._check(lib().tof_profile_burst_read(self._ctx, ms))
        return [ms[i] for i in range(PROFILE_SLOTS)]

    def profile_kernels(self, with_items: bool = False):
        """Per slot: the name of the kernel last timed there ("" if none), or
        (name, work items of that launch) with with_items."""
        out = []
        for i in range(PROFILE_SLOTS):
            n = ctypes.c_int64(0)
            name = lib().tof_profile_kernel(self._ctx, i, ctypes.byref(n)).decode()
            out.append((name, int(n.value)) if with_items else name)
        return out

    def set_option(self, option: int, value):
        """Pass choice (OPT_ZSUM, OPT_FUSE_YZ, OPT_FUSE_OBJECTIVE: a bool) or
        tile choice (OPT_X_TILE, OPT_GATHER_GROUPS, OPT_SCATTER_GROUPS: an
        int); see tof_set_option."""
        v = (1 if value else 0) if isinstance(value, bool) else int(value)
        self._check(lib().tof_set_option(self._ctx, int(option), v))

    def padded_lengths(self) -> Tuple[int, int, int]:
        out = (ctypes.c_int32 * 3)()
        self._check(lib().tof_padded_lengths(self._ctx, out))
        return tuple(out)

    def ctx_bytes(self) -> int:
        """Device bytes the context holds (tof_ctx_bytes)."""
        return int(lib().tof_ctx_bytes(self._ctx))


class Batch:
    """tof_batch: one gradient evaluation of many designs with one launch per
    pass and kernel instantiation (the engines' contexts and the rho, J, grad
    tensors are borrowed and kept referenced here)."""

    def __init__(self, engines, rho, J, grad):
        n = len(engines)
        vp = ctypes.c_void_p
        arr = lambda xs: (vp * n)(*[vp(x) for x in xs])
        self._refs = (list(engines), list(rho), list(J), list(grad))
        self._b = vp()
        for e, r, j, g in zip(engines, rho, J, grad):
            e._arr(r, e.shape)
            e._arr(g, e.shape)
            e._arr(j, (1,), e.torch.float64)
        st = lib().tof_batch_create(arr([e._ctx.value for e in engines]), arr([r.data_ptr() for r in rho]),
                                    arr([j.data_ptr() for j in J]), arr([g.data_ptr() for g in grad]), n,
                                    ctypes.byref(self._b))
        if st != 0:
            raise TofError(st, lib().tof_last_error(None).decode())

    def run(self, stream=None):
        st = lib().tof_batch_run(self._b, _stream_ptr(stream))
        if st != 0:
            raise TofError(st, lib().tof_last_error(None).decode())

    def launches(self) -> int:
        return int(lib().tof_batch_launches(self._b))

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib().tof_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_grid(n, h, dtype: str = "f32", L=None, validate: bool = False, flags: int = 0) -> Grid:
    Lx, Ly, Lz = (0, 0, 0) if L is None else (int(v) for v in L)
    return Grid(int(n[0]), int(n[1]), int(n[2]), float(h[0]), float(h[1]), float(h[2]), Lx, Ly, Lz,
                TOF_F32 if dtype == "f32" else TOF_F64, 1 if validate else 0, int(flags))


def workspace_bytes(n, h, dtype: str = "f32", L=None) -> int:
    """Device bytes a context for this grid holds after setup (tof_workspace_bytes;
    host arithmetic only, no device needed).  Raises on an invalid grid."""
    g = make_grid(n, h, dtype, L)
    b = int(lib().tof_workspace_bytes(ctypes.byref(g)))
    if b == 0:
        raise TofError(-1, lib().tof_last_error(None).decode())
    return b


def project_step_static(rho, grad, alpha: float, design=None, mask=None, stream=None):
    """tof_project_step_static: the projected step with no context and no
    allocation (rho [nz][ny][nx] is updated in place)."""
    import torch
    if rho.dtype not in (torch.float32, torch.float64) or rho.device.type != "cuda" or not rho.is_contiguous() \
            or rho.dim() != 3 or grad.shape != rho.shape or grad.dtype != rho.dtype or not grad.is_contiguous():
        raise ValueError("rho and grad must be contiguous 3-d cuda tensors of one float dtype")
    nz, ny, nx = (int(v) for v in rho.shape)
    g = make_grid((nx, ny, nz), (1.0, 1.0, 1.0), "f32" if rho.dtype == torch.float32 else "f64")
    bx = ctypes.byref(_box(design)) if design is not None else None
    mk = None
    if mask is not None:
        if mask.dtype != torch.uint8 or tuple(mask.shape) != tuple(rho.shape) or not mask.is_contiguous():
            raise ValueError("mask must be a contiguous uint8 tensor shaped like rho")
        mk = ctypes.c_void_p(mask.data_ptr())
    st = lib().tof_project_step_static(ctypes.byref(g), bx, mk, ctypes.c_void_p(rho.data_ptr()),
                                       ctypes.c_void_p(grad.data_ptr()), float(alpha), _stream_ptr(stream))
    if st != 0:
        raise TofError(st, lib().tof_last_error(None).decode())
    return rho


def engine_for(w, dtype: str = "f32", stream=None, L=None, validate: bool = False) -> Engine:
    """An Engine set up for a workload description (workloads.Workload); L
    overrides the workload's padded lengths."""
    import torch
    e = Engine(w.n, w.h, dtype, L=w.pad if L is None else L, stream=stream, validate=validate)
    tdt = e.dtype
    m0f = None
    if w.m0_field is not None:
        m0f = torch.as_tensor(w.m0_field, dtype=tdt).contiguous().cuda()
    mask = None
    if getattr(w, "mask", None) is not None:
        mask = torch.as_tensor(w.mask, dtype=torch.uint8).contiguous().cuda()
    e.set_design(w.design, m0=w.m0, m0_field=m0f, p=w.p, mask=mask)
    e.set_objective(w.j_kind, w.sensor, w.j_target, w.j_lambda, w.h_target)
    return e


def newell_host(c: int, k: Sequence[int], h: Sequence[float]) -> float:
    """The double-double tensor entry the GPU setup computes, evaluated on the host."""
    return float(lib().tof_dd_newell_host(int(c), int(k[0]), int(k[1]), int(k[2]),
                                          float(h[0]), float(h[1]), float(h[2])))
