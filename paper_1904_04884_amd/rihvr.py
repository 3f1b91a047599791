"""Python binding of librihvr.so (ctypes).

The functions `ri_*` mirror the C ABI one to one (argument marshalling only;
pointers are plain integers, streams are hipStream_t handles as integers).
`Plan` is a convenience wrapper that takes torch tensors: torch provides device
memory and the current stream, every computation runs in the HIP library.

Importing this module does not load the library; the first call does, and it
raises if the library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import math
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "librihvr.so"

# ---------------------------------------------------------------------------
# ABI types (layouts match include/rihvr.h)
# ---------------------------------------------------------------------------
RI_OK = 0
RI_ERR_INVALID_ARG = 1
RI_ERR_UNSUPPORTED_SIZE = 2
RI_ERR_OUT_OF_MEMORY = 3
RI_ERR_WORKSPACE_TOO_SMALL = 4
RI_ERR_HIP = 5
RI_ERR_NONFINITE = 6
RI_ERR_NOT_CONVERGED = 7

RI_F32, RI_F64 = 0, 1

RI_NO_CARRIER = 0x1
RI_TV2D = 0x2
RI_TV_FGP = 0x4
RI_TV_DUAL_BF16 = 0x8
RI_COMPLEX = 0x10
RI_INIT_ZERO = 0
RI_INIT_GIVEN = 1
RI_SOLVE_DENSE = 0x1
RI_SOLVE_NO_GRAPH = 0x2
RI_SOLVE_RESTART = 0x4
RI_SOLVE_TIMING = 0x8
RI_SOLVE_DUAL_WARM = 0x10
RI_SOLVE_GROUPED = 0x20

RI_OP_FORWARD, RI_OP_ADJOINT, RI_OP_PROX, RI_OP_SOLVE, RI_OP_AUTOTUNE = 0, 1, 2, 3, 4
RI_NUM_PHASES = 6
PHASE_NAMES = ("forward", "hologram", "adjoint", "prox", "objective", "other")

EXPORTED = (
    "ri_plan_create", "ri_plan_destroy", "ri_plan_lipschitz", "ri_workspace_size", "ri_workspace_size_op",
    "ri_plan_get_tuning", "ri_plan_set_tuning", "ri_plan_set_storage", "ri_plan_get_storage",
    "ri_plan_set_dual_planes", "ri_plan_get_dual_planes", "ri_plan_autotune",
    "ri_forward", "ri_forward_noalloc", "ri_forward_noalloc_max_scratch", "ri_adjoint", "ri_prox_fused_lasso", "ri_solve", "ri_solve_batched",
    "ri_workspace_size_batched",
    "ri_unet_param_count", "ri_unet_init_params", "ri_unet_workspace_size", "ri_unet_forward",
    "ri_unet_train_step",
    "ri_detect_workspace_size", "ri_detect", "ri_link_workspace_size", "ri_link", "ri_track_update",
    "ri_track_filter",
    "ri_status_string", "ri_last_error",
)


class ri_detect_params(C.Structure):
    _fields_ = [("rel_threshold", C.c_double), ("min_voxels", C.c_int32)]


RI_OBJECT_FIELDS = ("z", "y", "x", "weight", "voxels", "first")   # ri_object: 6 doubles


class ri_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("pixel_um", C.c_double), ("wavelength_um", C.c_double),
                ("z0_um", C.c_double), ("dz_um", C.c_double), ("flags", C.c_uint32)]


class ri_prox_params(C.Structure):
    _fields_ = [("l1", C.c_double), ("tv", C.c_double), ("inner_iters", C.c_int32), ("nonneg", C.c_int32)]


class ri_solve_params(C.Structure):
    _fields_ = [("l1", C.c_double), ("tv", C.c_double), ("max_iters", C.c_int32), ("inner_iters", C.c_int32),
                ("gap_tol", C.c_double), ("f_ref", C.c_double), ("init", C.c_int32),
                ("check_every", C.c_int32), ("flags", C.c_uint32), ("nonneg", C.c_int32),
                ("x0_scale", C.c_double)]


class ri_solve_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("objective", C.c_double),
                ("objective_min", C.c_double), ("gap", C.c_double),
                ("lipschitz", C.c_double), ("empty_plane_frac", C.c_double), ("empty_row_frac", C.c_double),
                ("phase_ms", C.c_double * RI_NUM_PHASES), ("phase_launches", C.c_int32 * RI_NUM_PHASES),
                ("store_rows_peak", C.c_int32)]

    def as_dict(self):
        return {
            "store_rows_peak": self.store_rows_peak,
            "iters": self.iters, "converged": bool(self.converged), "objective": self.objective,
            "objective_min": self.objective_min,
            "gap": self.gap, "lipschitz": self.lipschitz, "empty_plane_frac": self.empty_plane_frac,
            "empty_row_frac": self.empty_row_frac,
            "phase_ms": {n: self.phase_ms[i] for i, n in enumerate(PHASE_NAMES)},
            "phase_launches": {n: self.phase_launches[i] for i, n in enumerate(PHASE_NAMES)},
        }


class ri_tuning(C.Structure):
    _fields_ = [("tv_levels", C.c_int32), ("tv_blocks", C.c_int32), ("col_blocks", C.c_int32)]

    def as_dict(self):
        return {"tv_levels": self.tv_levels, "tv_blocks": self.tv_blocks, "col_blocks": self.col_blocks}


class ri_autotune_report(C.Structure):
    _fields_ = [("best", ri_tuning), ("from_cache", C.c_int32), ("cache_written", C.c_int32),
                ("candidates", C.c_int32), ("default_ms", C.c_double), ("best_ms", C.c_double),
                ("tune_ms", C.c_double)]

    def as_dict(self):
        return {"best": self.best.as_dict(), "from_cache": bool(self.from_cache),
                "cache_written": self.cache_written, "candidates": self.candidates,
                "default_ms": self.default_ms, "best_ms": self.best_ms, "tune_ms": self.tune_ms}


class ri_unet_config(C.Structure):
    _fields_ = [("levels", C.c_int32), ("base", C.c_int32)]


class RihvrError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def lib():
    """Load librihvr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_1904_04884_amd.build_lib`")
    L = C.CDLL(str(LIB_PATH))
    vp, sz = C.c_void_p, C.c_size_t
    L.ri_plan_create.argtypes = [C.POINTER(ri_geometry), C.c_int, C.POINTER(vp)]
    L.ri_plan_destroy.argtypes = [vp]
    L.ri_plan_lipschitz.argtypes = [vp, C.POINTER(C.c_double)]
    L.ri_workspace_size.argtypes = [vp, C.POINTER(sz)]
    L.ri_workspace_size_op.argtypes = [vp, C.c_int, C.POINTER(sz)]
    L.ri_plan_get_tuning.argtypes = [vp, C.POINTER(ri_tuning)]
    L.ri_plan_set_tuning.argtypes = [vp, C.POINTER(ri_tuning)]
    L.ri_plan_set_storage.argtypes = [vp, C.c_double]
    L.ri_plan_get_storage.argtypes = [vp, C.POINTER(C.c_double)]
    L.ri_plan_set_dual_planes.argtypes = [vp, C.c_int32]
    L.ri_plan_get_dual_planes.argtypes = [vp, C.POINTER(C.c_int32)]
    L.ri_plan_autotune.argtypes = [vp, C.c_int32, C.c_char_p, vp, sz, vp, C.POINTER(ri_autotune_report)]
    L.ri_forward.argtypes = [vp, vp, vp, vp, sz, vp]
    L.ri_forward_noalloc.argtypes = [vp, vp, vp, vp]
    L.ri_forward_noalloc_max_scratch.argtypes = []
    L.ri_adjoint.argtypes = [vp, vp, vp, vp, sz, vp]
    L.ri_prox_fused_lasso.argtypes = [vp, C.POINTER(ri_prox_params), C.c_double, vp, vp, vp, sz, vp]
    L.ri_solve.argtypes = [vp, C.POINTER(ri_solve_params), vp, vp, vp, sz, vp, C.POINTER(ri_solve_report)]
    L.ri_solve_batched.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(ri_solve_params), C.POINTER(vp),
                                   C.POINTER(vp), vp, sz, vp, C.POINTER(ri_solve_report)]
    L.ri_workspace_size_batched.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(ri_solve_params),
                                            C.POINTER(sz)]
    cfgp, fp = C.POINTER(ri_unet_config), C.c_float
    L.ri_unet_param_count.argtypes = [cfgp, C.POINTER(sz)]
    L.ri_unet_init_params.argtypes = [cfgp, C.c_uint64, vp, vp]
    L.ri_unet_workspace_size.argtypes = [cfgp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(sz)]
    L.ri_unet_forward.argtypes = [cfgp, vp, vp, fp, vp, C.c_int32, C.c_int32, C.c_int32, vp, sz, vp]
    L.ri_unet_train_step.argtypes = [cfgp, vp, vp, vp, vp, C.c_int32, fp, vp, fp, vp, fp, C.c_int32, C.c_int32,
                                     C.c_int32, vp, vp, sz, vp]
    L.ri_forward_noalloc_max_scratch.restype = C.c_size_t
    i32 = C.c_int32
    L.ri_detect_workspace_size.argtypes = [i32, i32, i32, i32, C.POINTER(C.c_size_t)]
    L.ri_detect.argtypes = [C.POINTER(ri_detect_params), vp, i32, i32, i32, vp, i32, vp, i32, vp, sz, vp]
    L.ri_link_workspace_size.argtypes = [i32, i32, C.POINTER(C.c_size_t)]
    L.ri_link.argtypes = [vp, vp, i32, vp, vp, i32, C.POINTER(C.c_double), C.c_double, vp, vp, vp, sz, vp]
    L.ri_track_update.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, i32, vp]
    L.ri_track_filter.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.ri_status_string.argtypes = [C.c_int]
    L.ri_status_string.restype = C.c_char_p
    L.ri_last_error.argtypes = []
    L.ri_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("ri_status_string", "ri_last_error", "ri_forward_noalloc_max_scratch"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int, where: str):
    if status != RI_OK:
        L = lib()
        raise RihvrError(status, where, f"{L.ri_status_string(status).decode()}: {L.ri_last_error().decode()}")


# ---------------------------------------------------------------------------
# One-to-one wrappers (raw pointers as ints)
# ---------------------------------------------------------------------------
def ri_plan_create(geometry: ri_geometry, dtype: int = RI_F32) -> int:
    h = C.c_void_p()
    _check(lib().ri_plan_create(C.byref(geometry), int(dtype), C.byref(h)), "ri_plan_create")
    return h.value


def ri_plan_destroy(plan: int) -> None:
    _check(lib().ri_plan_destroy(plan), "ri_plan_destroy")


def ri_plan_lipschitz(plan: int) -> float:
    v = C.c_double()
    _check(lib().ri_plan_lipschitz(plan, C.byref(v)), "ri_plan_lipschitz")
    return v.value


def ri_workspace_size(plan: int) -> int:
    v = C.c_size_t()
    _check(lib().ri_workspace_size(plan, C.byref(v)), "ri_workspace_size")
    return v.value


def ri_workspace_size_op(plan: int, op: int) -> int:
    v = C.c_size_t()
    _check(lib().ri_workspace_size_op(plan, op, C.byref(v)), "ri_workspace_size_op")
    return v.value


def ri_plan_get_tuning(plan: int) -> ri_tuning:
    t = ri_tuning()
    _check(lib().ri_plan_get_tuning(plan, C.byref(t)), "ri_plan_get_tuning")
    return t


def ri_plan_set_tuning(plan: int, tuning: ri_tuning) -> int:
    return lib().ri_plan_set_tuning(plan, C.byref(tuning))


def ri_plan_set_storage(plan: int, row_fraction: float) -> int:
    return lib().ri_plan_set_storage(plan, float(row_fraction))


def ri_plan_get_storage(plan: int) -> float:
    v = C.c_double()
    _check(lib().ri_plan_get_storage(plan, C.byref(v)), "ri_plan_get_storage")
    return v.value


def ri_plan_set_dual_planes(plan: int, planes: int) -> int:
    return lib().ri_plan_set_dual_planes(plan, int(planes))


def ri_plan_get_dual_planes(plan: int) -> int:
    v = C.c_int32()
    _check(lib().ri_plan_get_dual_planes(plan, C.byref(v)), "ri_plan_get_dual_planes")
    return v.value


def ri_plan_autotune(plan, inner_iters, cache_path, ws, ws_bytes, stream, report=None) -> int:
    path = None if cache_path is None else str(cache_path).encode()
    return lib().ri_plan_autotune(plan, inner_iters, path, ws, ws_bytes, stream,
                                  C.byref(report) if report is not None else None)


def ri_forward(plan, x, b_out, ws, ws_bytes, stream) -> int:
    return lib().ri_forward(plan, x, b_out, ws, ws_bytes, stream)


def ri_forward_noalloc(plan, x, b_out, stream) -> int:
    return lib().ri_forward_noalloc(plan, x, b_out, stream)


def ri_forward_noalloc_max_scratch() -> int:
    return int(lib().ri_forward_noalloc_max_scratch())


def ri_adjoint(plan, y, x_out, ws, ws_bytes, stream) -> int:
    return lib().ri_adjoint(plan, y, x_out, ws, ws_bytes, stream)


def ri_prox_fused_lasso(plan, params: ri_prox_params, step, v, x_out, ws, ws_bytes, stream) -> int:
    return lib().ri_prox_fused_lasso(plan, C.byref(params), step, v, x_out, ws, ws_bytes, stream)


def ri_solve(plan, params: ri_solve_params, b, x_inout, ws, ws_bytes, stream, report=None) -> int:
    return lib().ri_solve(plan, C.byref(params), b, x_inout, ws, ws_bytes, stream,
                          C.byref(report) if report is not None else None)


def ri_solve_batched(n, plans, params, b, x_inout, ws, ws_bytes, stream, reports=None) -> int:
    P = (C.c_void_p * n)(*plans)
    Q = (ri_solve_params * n)(*params)
    B = (C.c_void_p * n)(*b)
    X = (C.c_void_p * n)(*x_inout)
    return lib().ri_solve_batched(n, P, Q, B, X, ws, ws_bytes, stream, reports)


def ri_workspace_size_batched(n, plans, params) -> int:
    P = (C.c_void_p * n)(*plans)
    Q = (ri_solve_params * n)(*params)
    v = C.c_size_t()
    _check(lib().ri_workspace_size_batched(n, P, Q, C.byref(v)), "ri_workspace_size_batched")
    return v.value


def ri_unet_param_count(cfg: ri_unet_config) -> int:
    v = C.c_size_t()
    _check(lib().ri_unet_param_count(C.byref(cfg), C.byref(v)), "ri_unet_param_count")
    return v.value


def ri_unet_init_params(cfg, seed, params, stream) -> int:
    return lib().ri_unet_init_params(C.byref(cfg), seed, params, stream)


def ri_unet_workspace_size(cfg, d, h, w, training) -> int:
    v = C.c_size_t()
    _check(lib().ri_unet_workspace_size(C.byref(cfg), d, h, w, training, C.byref(v)), "ri_unet_workspace_size")
    return v.value


def ri_unet_forward(cfg, params, inp, scale, out, d, h, w, ws, ws_bytes, stream) -> int:
    return lib().ri_unet_forward(C.byref(cfg), params, inp, scale, out, d, h, w, ws, ws_bytes, stream)


def ri_unet_train_step(cfg, params, grads, m, v, step, lr, inp, scale, target, pos_weight, d, h, w, loss, ws,
                       ws_bytes, stream) -> int:
    return lib().ri_unet_train_step(C.byref(cfg), params, grads, m, v, step, lr, inp, scale, target, pos_weight,
                                    d, h, w, loss, ws, ws_bytes, stream)


def ri_status_string(status: int) -> str:
    return lib().ri_status_string(status).decode()


def ri_last_error() -> str:
    return lib().ri_last_error().decode()


# ---------------------------------------------------------------------------
# torch convenience layer
# ---------------------------------------------------------------------------
def _stream_handle(torch):
    return torch.cuda.current_stream().cuda_stream


def geometry_struct(geom) -> ri_geometry:
    """From any object with nx, ny, nz, pixel_um, wavelength_um, z0_um, dz_um[, carrier, tv_dims]."""
    flags = 0 if getattr(geom, "carrier", True) else RI_NO_CARRIER
    if getattr(geom, "tv_dims", 3) == 2:
        flags |= RI_TV2D
    if getattr(geom, "tv_fgp", False):
        flags |= RI_TV_FGP
    if getattr(geom, "dual_bf16", False):
        flags |= RI_TV_DUAL_BF16
    if getattr(geom, "complex_object", False):
        flags |= RI_COMPLEX
    return ri_geometry(int(geom.nx), int(geom.ny), int(geom.nz), float(geom.pixel_um),
                       float(geom.wavelength_um), float(geom.z0_um), float(geom.dz_um), flags)


class Plan:
    """A plan plus lazily allocated (torch) workspaces for one geometry.
    dtype RI_F64: every array argument is float64 (the FP64 path)."""

    def __init__(self, geom, dtype=RI_F32):
        import torch
        self.torch = torch
        self.geom = geom
        self.dtype = int(dtype)
        self.tdtype = torch.float64 if self.dtype == RI_F64 else torch.float32
        self.handle = ri_plan_create(geometry_struct(geom), self.dtype)
        self.lipschitz = ri_plan_lipschitz(self.handle)
        self._ws = {}

    def close(self):
        if self.handle:
            ri_plan_destroy(self.handle)
            self.handle = None
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        """Shape of a volume argument: [nz][ny][nx], or [2][nz][ny][nx] (real
        parts, imaginary parts) for a complex object."""
        if getattr(self.geom, "complex_object", False):
            return (2, self.geom.nz, self.geom.ny, self.geom.nx)
        return (self.geom.nz, self.geom.ny, self.geom.nx)

    def workspace(self, op: int):
        n = ri_workspace_size_op(self.handle, op)
        ws = self._ws.get(op)
        if ws is None or ws.numel() < n:
            ws = self.torch.empty(max(n, 1), dtype=self.torch.uint8, device="cuda")
            self._ws[op] = ws
        return ws, n

    @property
    def tuning(self) -> dict:
        return ri_plan_get_tuning(self.handle).as_dict()

    @tuning.setter
    def tuning(self, t: dict):
        _check(ri_plan_set_tuning(self.handle, ri_tuning(int(t["tv_levels"]), int(t["tv_blocks"]),
                                                         int(t["col_blocks"]))), "ri_plan_set_tuning")

    @property
    def dual_planes(self) -> int:
        """Planes whose TV dual the per-plane prox holds at a time (0: all; see
        ri_plan_set_dual_planes)."""
        return ri_plan_get_dual_planes(self.handle)

    @dual_planes.setter
    def dual_planes(self, n: int):
        _check(ri_plan_set_dual_planes(self.handle, n), "ri_plan_set_dual_planes")

    @property
    def row_fraction(self) -> float:
        """Storage of the solver's iterates: 0 dense, else the fraction of rows
        each row store holds (see ri_plan_set_storage)."""
        return ri_plan_get_storage(self.handle)

    @row_fraction.setter
    def row_fraction(self, f: float):
        _check(ri_plan_set_storage(self.handle, f), "ri_plan_set_storage")

    def autotune(self, inner_iters: int, cache_path=None) -> dict:
        """Time the candidate launch shapes on the device and keep the fastest (see ri_plan_autotune)."""
        ws, n = self.workspace(RI_OP_AUTOTUNE)
        rep = ri_autotune_report()
        _check(ri_plan_autotune(self.handle, int(inner_iters), cache_path, ws.data_ptr(), ws.numel(),
                                _stream_handle(self.torch), rep), "ri_plan_autotune")
        self._ws.pop(RI_OP_AUTOTUNE, None)
        return rep.as_dict()

    def _chk(self, t, shape):
        torch = self.torch
        if not (t.is_cuda and t.dtype == self.tdtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected contiguous {self.tdtype} cuda tensor of shape {shape}, got "
                             f"{tuple(t.shape)} {t.dtype} {t.device}")

    def forward(self, x, out=None):
        torch = self.torch
        g = self.geom
        self._chk(x, self.shape)
        out = torch.empty((g.ny, g.nx), dtype=self.tdtype, device="cuda") if out is None else out
        ws, n = self.workspace(RI_OP_FORWARD)
        _check(ri_forward(self.handle, x.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                          _stream_handle(torch)), "ri_forward")
        return out

    def adjoint(self, y, out=None):
        torch = self.torch
        self._chk(y, (self.geom.ny, self.geom.nx))
        out = torch.empty(self.shape, dtype=self.tdtype, device="cuda") if out is None else out
        ws, n = self.workspace(RI_OP_ADJOINT)
        _check(ri_adjoint(self.handle, y.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                          _stream_handle(torch)), "ri_adjoint")
        return out

    def prox(self, v, step, l1, tv, inner_iters, nonneg=True, out=None):
        torch = self.torch
        self._chk(v, self.shape)
        out = torch.empty_like(v) if out is None else out
        ws, n = self.workspace(RI_OP_PROX)
        p = ri_prox_params(float(l1), float(tv), int(inner_iters), 1 if nonneg else 0)
        _check(ri_prox_fused_lasso(self.handle, p, float(step), v.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream_handle(torch)), "ri_prox_fused_lasso")
        return out

    def solve_params(self, l1, tv, max_iters, inner_iters, gap_tol=0.0, f_ref=0.0, init=RI_INIT_ZERO,
                     check_every=10, flags=0, nonneg=True, x0_scale=1.0) -> ri_solve_params:
        return ri_solve_params(float(l1), float(tv), int(max_iters), int(inner_iters), float(gap_tol),
                               float(f_ref), int(init), int(check_every), int(flags), 1 if nonneg else 0,
                               float(x0_scale))

    def solve(self, b, l1, tv, max_iters, inner_iters, x=None, gap_tol=0.0, f_ref=0.0, check_every=10,
              flags=0, nonneg=True, report=True, raise_on_error=True, x0_scale=1.0):
        torch = self.torch
        self._chk(b, (self.geom.ny, self.geom.nx))
        init = RI_INIT_ZERO
        if x is None:
            x = torch.empty(self.shape, dtype=self.tdtype, device="cuda")
        else:
            self._chk(x, self.shape)
            init = RI_INIT_GIVEN
        ws, n = self.workspace(RI_OP_SOLVE)
        sp = self.solve_params(l1, tv, max_iters, inner_iters, gap_tol, f_ref, init, check_every, flags, nonneg,
                               x0_scale)
        rep = ri_solve_report() if report else None
        st = ri_solve(self.handle, sp, b.data_ptr(), x.data_ptr(), ws.data_ptr(), ws.numel(),
                      _stream_handle(torch), rep)
        if raise_on_error:
            _check(st, "ri_solve")
        return x, (rep.as_dict() if rep is not None else None), st


def objective_gap(f, f_ref):
    return (f - f_ref) / f_ref if f_ref > 0 else math.nan


class UNet:
    """Warm-start network with FP32 parameters and Adam moments in torch tensors."""

    def __init__(self, levels=4, base=16, seed=0):
        import torch
        self.torch = torch
        self.cfg = ri_unet_config(int(levels), int(base))
        self.n = ri_unet_param_count(self.cfg)
        self.params = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = None
        _check(ri_unet_init_params(self.cfg, int(seed), self.params.data_ptr(), _stream_handle(torch)),
               "ri_unet_init_params")

    def _workspace(self, d, h, w, training):
        n = ri_unet_workspace_size(self.cfg, d, h, w, 1 if training else 0)
        if self._ws is None or self._ws.numel() < n:
            self._ws = self.torch.empty(n, dtype=self.torch.uint8, device="cuda")
        return self._ws

    def forward(self, inp, scale=1.0, out=None):
        torch = self.torch
        d, h, w = inp.shape
        out = torch.empty_like(inp) if out is None else out
        ws = self._workspace(d, h, w, False)
        _check(ri_unet_forward(self.cfg, self.params.data_ptr(), inp.data_ptr(), float(scale), out.data_ptr(),
                               d, h, w, ws.data_ptr(), ws.numel(), _stream_handle(torch)), "ri_unet_forward")
        return out

    def train_step(self, inp, target, lr=1e-3, scale=1.0, pos_weight=1.0):
        torch = self.torch
        d, h, w = inp.shape
        ws = self._workspace(d, h, w, True)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        if lr > 0:
            self.step += 1
        _check(ri_unet_train_step(self.cfg, self.params.data_ptr(), self.grads.data_ptr(), self.m.data_ptr(),
                                  self.v.data_ptr(), max(self.step, 1), float(lr), inp.data_ptr(), float(scale),
                                  target.data_ptr(), float(pos_weight), d, h, w, loss.data_ptr(), ws.data_ptr(),
                                  ws.numel(),
                                  _stream_handle(torch)), "ri_unet_train_step")
        return loss


# ---------------------------------------------------------------------------
# Particle tracking back end (torch tensors in, torch tensors out)
# ---------------------------------------------------------------------------
def detect(x, rel_threshold=1.0 / 256.0, min_voxels=5, max_objects=65536, max_components=1 << 20):
    """Objects of a float32 volume [nz][ny][nx] on the device: returns
    (objects [max_objects][6] float64 device tensor, counts [2] int32 device
    tensor: kept objects, components).  Rows follow ri_object (z, y, x,
    weight, voxels, first)."""
    import torch
    nz, ny, nx = x.shape
    nbytes = C.c_size_t()
    _check(lib().ri_detect_workspace_size(nx, ny, nz, max_components, C.byref(nbytes)), "ri_detect_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=x.device)
    objs = torch.zeros((max_objects, 6), dtype=torch.float64, device=x.device)
    counts = torch.zeros(2, dtype=torch.int32, device=x.device)
    prm = ri_detect_params(float(rel_threshold), int(min_voxels))
    _check(lib().ri_detect(C.byref(prm), x.data_ptr(), nx, ny, nz, objs.data_ptr(), max_objects, counts.data_ptr(),
                           max_components, ws.data_ptr(), ws.numel(), _stream_handle(torch)), "ri_detect")
    return objs, counts


def link(prev, n_prev, cur, n_cur, max_disp, spacing=(1.0, 1.0, 1.0)):
    """Crocker-Grier links of object tables prev -> cur (device tensors with
    device counts n_prev, n_cur: int32 tensors of one element): returns
    (link [len(prev)] int32, status [1] int32), both on the device."""
    import torch
    nbytes = C.c_size_t()
    _check(lib().ri_link_workspace_size(prev.shape[0], cur.shape[0], C.byref(nbytes)), "ri_link_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=prev.device)
    lk = torch.full((prev.shape[0],), -1, dtype=torch.int32, device=prev.device)
    status = torch.zeros(1, dtype=torch.int32, device=prev.device)
    sp = (C.c_double * 3)(*[float(v) for v in spacing])
    _check(lib().ri_link(prev.data_ptr(), n_prev.data_ptr(), prev.shape[0], cur.data_ptr(), n_cur.data_ptr(),
                         cur.shape[0], sp, float(max_disp), lk.data_ptr(), status.data_ptr(), ws.data_ptr(),
                         ws.numel(), _stream_handle(torch)), "ri_link")
    return lk, status


class Tracks:
    """Track ids frame by frame on the device (ri_track_update), then the
    minimum-duration filter (ri_track_filter)."""

    def __init__(self, max_tracks=1 << 20):
        import torch
        self.torch = torch
        self.max_tracks = max_tracks
        self.track_len = torch.zeros(max_tracks, dtype=torch.int32, device="cuda")
        self.next_id = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.ids = None
        self.n = torch.zeros(1, dtype=torch.int32, device="cuda")

    def update(self, lk, n_cur, max_cur):
        """lk: links from the previous frame (None for the first frame)."""
        torch = self.torch
        ids = torch.full((max_cur,), -1, dtype=torch.int32, device="cuda")
        zero = torch.zeros(1, dtype=torch.int32, device="cuda")
        n_prev = self.n if lk is not None else zero
        _check(lib().ri_track_update(lk.data_ptr() if lk is not None else None, n_prev.data_ptr(),
                                     self.ids.data_ptr() if lk is not None else None, n_cur.data_ptr(), max_cur,
                                     ids.data_ptr(), self.next_id.data_ptr(), self.track_len.data_ptr(),
                                     self.max_tracks, _stream_handle(torch)), "ri_track_update")
        self.ids = ids
        self.n = n_cur.clone()
        return ids

    def kept(self, min_len):
        torch = self.torch
        kept = torch.zeros(self.max_tracks, dtype=torch.uint8, device="cuda")
        n_kept = torch.zeros(1, dtype=torch.int32, device="cuda")
        _check(lib().ri_track_filter(self.track_len.data_ptr(), self.next_id.data_ptr(), self.max_tracks,
                                     int(min_len), kept.data_ptr(), n_kept.data_ptr(), _stream_handle(torch)),
               "ri_track_filter")
        return kept, n_kept
