"""Thin Python binding of the C ABI in include/ell.h.

Argument marshalling only: every step of the solver runs in the HIP kernels
of libell.so.  PyTorch provides device memory (tensors) and the stream; the
library and PyTorch share one HIP runtime (torch is imported first, so the
runtime it loaded also serves libell.so).

If the library has not been built this module raises ImportError: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ELL_LIBRARY", os.path.join(HERE, "libell.so"))

ELL_OK, ELL_NOT_CONVERGED, ELL_PENDING = 0, 1, 2
ELL_ERR_INVALID, ELL_ERR_OOM, ELL_ERR_HIP, ELL_ERR_NUMERIC, ELL_ERR_BUDGET = -1, -2, -3, -4, -5
ELL_FP64, ELL_FP32_PRECOND, ELL_FP32_BF16COEF = 0, 1, 2
PRECISIONS = {"fp64": ELL_FP64, "fp32": ELL_FP32_PRECOND, "bf16coef": ELL_FP32_BF16COEF}
ELL_K_SMOOTH0, ELL_K_APPLY, ELL_K_RESTRICT0, ELL_K_PROLONG0, ELL_K_UPDATE, ELL_K_COUNT = 0, 1, 2, 3, 4, 5

_dp = ctypes.POINTER(ctypes.c_double)


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("omega2", ctypes.c_double),
                ("dz", _dp), ("lambda2", _dp), ("n_levels", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("nu_coarse", ctypes.c_int32), ("rho", ctypes.c_double),
                ("prolong", ctypes.c_int32), ("precision", ctypes.c_int32)]


ELL_MAX_LEVELS = 16


class Schedule(ctypes.Structure):
    _fields_ = [("apply_tile", ctypes.c_int32), ("apply_nseg", ctypes.c_int32),
                ("smooth_nseg", ctypes.c_int32 * ELL_MAX_LEVELS), ("ms_per_iter", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("maxiter", ctypes.c_int32),
                ("flexible", ctypes.c_int32), ("rel_to_rhs", ctypes.c_int32),
                ("poll_every", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("r0_norm", ctypes.c_double),
                ("r_norm", ctypes.c_double), ("true_r_norm", ctypes.c_double),
                ("b_norm", ctypes.c_double)]


EXPORTS = ["ell_grid_create", "ell_grid_destroy", "ell_grid_bytes", "ell_grid_levels", "ell_grid_features",
           "ell_apply_A", "ell_vcycle", "ell_pcg_solve", "ell_level_elems", "ell_to_split",
           "ell_from_split", "ell_level_smooth", "ell_level_resid_restrict",
           "ell_level_prolong_add", "ell_level_apply", "ell_profile_enable", "ell_profile_pause", "ell_profile_read",
           "ell_profile_times", "ell_level_layout", "ell_set_tuning", "ell_last_error",
           "ell_batch_create", "ell_batch_grid", "ell_batch_release", "ell_batch_bytes_in_use",
           "ell_batch_submit", "ell_batch_poll", "ell_batch_wait", "ell_batch_destroy",
           "ell_autotune", "ell_schedule_get", "ell_schedule_set", "ell_mg_solve",
           "ell_apply_A_noalloc", "ell_grid_create_varying"]
ELL_NOALLOC_MAX_NZ = 1024

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libell.so (does not initialise the GPU)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1307_2036_amd/build.py "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    L.ell_grid_create.argtypes = [ctypes.POINTER(GridDesc), ctypes.POINTER(vp)]
    L.ell_grid_create_varying.argtypes = [ctypes.POINTER(GridDesc), _dp, ctypes.POINTER(vp)]
    L.ell_grid_destroy.argtypes = [vp]
    L.ell_grid_bytes.argtypes = [ctypes.POINTER(GridDesc)]
    L.ell_grid_bytes.restype = ctypes.c_size_t
    L.ell_grid_levels.argtypes = [vp]
    L.ell_grid_features.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.ell_apply_A.argtypes = [vp, vp, vp, vp]
    L.ell_apply_A_noalloc.argtypes = [ctypes.POINTER(GridDesc), vp, vp, vp]
    L.ell_vcycle.argtypes = [vp, vp, vp, vp]
    L.ell_pcg_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
    L.ell_mg_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
    L.ell_level_elems.argtypes = [vp, i32]
    L.ell_level_elems.restype = ctypes.c_size_t
    L.ell_to_split.argtypes = [vp, i32, vp, vp, vp]
    L.ell_from_split.argtypes = [vp, i32, vp, vp, vp]
    L.ell_level_smooth.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    L.ell_level_resid_restrict.argtypes = [vp, i32, vp, vp, vp, i32, vp]
    L.ell_level_prolong_add.argtypes = [vp, i32, vp, vp, i32, vp]
    L.ell_level_apply.argtypes = [vp, i32, vp, vp, vp]
    L.ell_profile_enable.argtypes = [vp, i32, i32]
    L.ell_profile_pause.argtypes = [vp, i32, i32]
    L.ell_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    L.ell_profile_times.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_float), i32]
    L.ell_level_layout.argtypes = [vp, i32] + [ctypes.POINTER(ctypes.c_int64)] * 3
    L.ell_set_tuning.argtypes = [i32, i32]
    L.ell_last_error.restype = ctypes.c_char_p
    L.ell_batch_create.argtypes = [ctypes.c_size_t, ctypes.POINTER(vp)]
    L.ell_batch_grid.argtypes = [vp, ctypes.POINTER(GridDesc), ctypes.POINTER(vp)]
    L.ell_batch_release.argtypes = [vp, vp]
    L.ell_batch_bytes_in_use.argtypes = [vp]
    L.ell_batch_bytes_in_use.restype = ctypes.c_size_t
    L.ell_batch_submit.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), ctypes.POINTER(SolveOpts),
                                   ctypes.POINTER(ctypes.c_uint64)]
    L.ell_batch_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(SolveStats)]
    L.ell_batch_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(SolveStats)]
    L.ell_batch_destroy.argtypes = [vp]
    L.ell_autotune.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_int32, ctypes.POINTER(Schedule)]
    L.ell_schedule_get.argtypes = [ctypes.POINTER(GridDesc), ctypes.POINTER(Schedule)]
    L.ell_schedule_set.argtypes = [ctypes.POINTER(GridDesc), ctypes.POINTER(Schedule)]
    for name in EXPORTS:
        if name not in ("ell_grid_bytes", "ell_level_elems", "ell_last_error", "ell_batch_bytes_in_use"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class EllError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ell error {code}: {msg}")
        self.code = code


def _check(rc: int, allow=(ELL_OK,)) -> int:
    if rc not in allow:
        raise EllError(rc, load_library().ell_last_error().decode())
    return rc


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype=torch.float64) -> ctypes.c_void_p:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_desc(nx, ny, nz, hx, hy, omega2, dz, lambda2, n_levels=0, nu_pre=1, nu_post=1,
              nu_coarse=1, rho=1.0, prolong=0, precision="fp64"):
    dz = np.ascontiguousarray(np.asarray(dz, dtype=np.float64))
    lam = np.ascontiguousarray(np.asarray(lambda2, dtype=np.float64))
    if dz.shape != (nz,) or lam.shape != (nz,):
        raise ValueError("dz and lambda2 must have nz entries")
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d = GridDesc(nx, ny, nz, hx, hy, omega2, dz.ctypes.data_as(_dp), lam.ctypes.data_as(_dp),
                 n_levels, nu_pre, nu_post, nu_coarse, rho, prolong, prec)
    return d, (dz, lam)


ELL_TUNE_PLANE_PAD, ELL_TUNE_COLOUR_PAD, ELL_TUNE_STENCIL_SEG, ELL_TUNE_APPLY_TILE = 0, 1, 2, 3
ELL_TUNE_BATCH_GRAPH = 4
ELL_TUNE_SMOOTH_TILE = 5
ELL_TUNE_FUSED_DOT = 6
ELL_TUNE_FUSED_UPDATE = 7
ELL_TUNE_FUSED_PROLONG = 8
ELL_TUNE_TILED_ENDS = 9
ELL_TUNE_COARSE_TAIL = 10
ELL_TUNE_COARSE_PAIR = 11
ELL_FEAT_TILED_SMOOTH, ELL_FEAT_FUSED_DOTS, ELL_FEAT_FUSED_UPDATE, ELL_FEAT_FUSED_PROLONG = 1, 2, 4, 8
ELL_FEAT_TILED_ENDS = 16
ELL_FEAT_COARSE_TAIL = 32
ELL_FEAT_COARSE_PROLONG = 64
ELL_FEAT_COARSE_PAIR = 128


def set_tuning(key: int, value: int) -> None:
    """Set one process-wide tuning key (ELL_TUNE_*: layout padding, kernel
    choices and fused forms) for grids and batches created afterwards."""
    _check(load_library().ell_set_tuning(key, value))


def _sched_dict(s: Schedule) -> dict:
    seg = list(s.smooth_nseg)
    while seg and seg[-1] == 0:
        seg.pop()
    return {"apply_tile": s.apply_tile, "apply_nseg": s.apply_nseg, "smooth_nseg": seg,
            "ms_per_iter": s.ms_per_iter}


def autotune(iters: int = 4, **desc) -> dict:
    """Time candidate schedules for this grid shape, record and return the
    fastest (see ell_autotune in ell.h)."""
    d, keep = make_desc(**desc)
    s = Schedule()
    _check(load_library().ell_autotune(ctypes.byref(d), iters, ctypes.byref(s)))
    return _sched_dict(s)


def schedule_get(**desc) -> dict:
    """The schedule a grid of this shape would get now."""
    d, keep = make_desc(**desc)
    s = Schedule()
    _check(load_library().ell_schedule_get(ctypes.byref(d), ctypes.byref(s)))
    return _sched_dict(s)


def schedule_set(schedule: Optional[dict], **desc) -> None:
    """Record a schedule for this shape (None clears the record)."""
    d, keep = make_desc(**desc)
    if schedule is None:
        _check(load_library().ell_schedule_set(ctypes.byref(d), None))
        return
    s = Schedule()
    s.apply_tile = int(schedule["apply_tile"])
    s.apply_nseg = int(schedule["apply_nseg"])
    for i, v in enumerate(schedule.get("smooth_nseg", [])):
        s.smooth_nseg[i] = int(v)
    _check(load_library().ell_schedule_set(ctypes.byref(d), ctypes.byref(s)))


def apply_A_noalloc(x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None, **desc) -> torch.Tensor:
    """y = A x for the grid described by ``desc`` (make_desc's arguments)
    without a grid object and without device allocation in the library
    (ell_apply_A_noalloc); x, y plane-major float64 CUDA tensors."""
    d, keep = make_desc(**desc)
    if y is None:
        y = torch.empty_like(x)
    _check(load_library().ell_apply_A_noalloc(ctypes.byref(d), _dev(x), _dev(y), _stream(stream)))
    return y


def grid_bytes(**kw) -> int:
    d, keep = make_desc(**kw)
    return int(load_library().ell_grid_bytes(ctypes.byref(d)))


@dataclass
class Stats:
    iters: int
    status: int
    r0_norm: float
    r_norm: float
    true_r_norm: float
    b_norm: float


class Grid:
    """Device-resident grid, multigrid hierarchy and solver workspace."""

    def __init__(self, nx, ny, nz, hx, hy, omega2, dz, lambda2, n_levels=0, nu_pre=1, nu_post=1,
                 nu_coarse=1, rho=1.0, prolong=0, precision="fp64", lambda2_3d=None):
        """lambda2_3d: None, or a (nz, ny, nx) field of lambda^2 cell values that
        replaces lambda2 (ell_grid_create_varying)."""
        L = load_library()
        d, keep = make_desc(nx, ny, nz, hx, hy, omega2, dz, lambda2, n_levels, nu_pre, nu_post,
                            nu_coarse, rho, prolong, precision)
        h = ctypes.c_void_p()
        if lambda2_3d is None:
            _check(L.ell_grid_create(ctypes.byref(d), ctypes.byref(h)))
        else:
            lam3 = np.ascontiguousarray(np.asarray(lambda2_3d, dtype=np.float64))
            if lam3.shape != (nz, ny, nx):
                raise ValueError("lambda2_3d must have shape (nz, ny, nx)")
            _check(L.ell_grid_create_varying(ctypes.byref(d), lam3.ctypes.data_as(_dp), ctypes.byref(h)))
        self.varying = lambda2_3d is not None
        self._h = h
        self.nx, self.ny, self.nz = nx, ny, nz
        self.precision = d.precision
        self.levels = L.ell_grid_levels(h)
        self.bytes = int(L.ell_grid_bytes(ctypes.byref(d)))
        m = ctypes.c_int32(0)
        _check(L.ell_grid_features(h, ctypes.byref(m)))
        self.features = {"tiled_smooth": bool(m.value & ELL_FEAT_TILED_SMOOTH),
                         "fused_dots": bool(m.value & ELL_FEAT_FUSED_DOTS),
                         "fused_update": bool(m.value & ELL_FEAT_FUSED_UPDATE),
                         "fused_prolong": bool(m.value & ELL_FEAT_FUSED_PROLONG),
                         "coarse_prolong": bool(m.value & ELL_FEAT_COARSE_PROLONG),
                         "coarse_pair": bool(m.value & ELL_FEAT_COARSE_PAIR),
                         "tiled_ends": bool(m.value & ELL_FEAT_TILED_ENDS),
                         "coarse_tail": bool(m.value & ELL_FEAT_COARSE_TAIL)}

    def feature_mask(self) -> int:
        """The current ell_grid_features mask (ELL_FEAT_*)."""
        m = ctypes.c_int32(0)
        _check(load_library().ell_grid_features(self._h, ctypes.byref(m)))
        return m.value

    @classmethod
    def from_problem(cls, p, precision="fp64", **over):
        kw = dict(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, omega2=p.omega2, dz=p.dz,
                  lambda2=p.lambda2, n_levels=p.n_levels, nu_pre=p.nu_pre, nu_post=p.nu_post,
                  nu_coarse=p.nu_coarse, rho=p.rho, prolong=p.prolong, precision=precision,
                  lambda2_3d=getattr(p, "lambda2_3d", None))
        kw.update(over)
        return cls(**kw)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ell_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def elem_dtype(self):
        return torch.float64 if self.precision == ELL_FP64 else torch.float32

    # ---- whole-path entry points -------------------------------------------------
    def apply_A(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None):
        y = torch.empty_like(x) if y is None else y
        _check(load_library().ell_apply_A(self._h, _dev(x), _dev(y), _stream(stream)))
        return y

    def vcycle(self, r: torch.Tensor, z: Optional[torch.Tensor] = None, stream=None):
        z = torch.empty_like(r) if z is None else z
        _check(load_library().ell_vcycle(self._h, _dev(r), _dev(z), _stream(stream)))
        return z

    def pcg_solve(self, f: torch.Tensor, u: Optional[torch.Tensor] = None, rtol=1e-5, atol=0.0,
                  maxiter=500, flexible=True, rel_to_rhs=False, poll_every=4, stream=None,
                  check=True):
        u = torch.zeros_like(f) if u is None else u
        o = SolveOpts(rtol, atol, maxiter, int(flexible), int(rel_to_rhs), poll_every)
        st = SolveStats()
        rc = load_library().ell_pcg_solve(self._h, _dev(f), _dev(u), ctypes.byref(o),
                                          ctypes.byref(st), _stream(stream))
        if check:
            _check(rc, allow=(ELL_OK, ELL_NOT_CONVERGED))
        return u, Stats(st.iters, st.status, st.r0_norm, st.r_norm, st.true_r_norm, st.b_norm)

    def mg_solve(self, f: torch.Tensor, u: Optional[torch.Tensor] = None, rtol=1e-5, atol=0.0,
                 maxiter=500, rel_to_rhs=False, poll_every=4, stream=None, check=True):
        """Stand-alone multigrid: repeated V-cycles (see ell_mg_solve)."""
        u = torch.zeros_like(f) if u is None else u
        o = SolveOpts(rtol, atol, maxiter, 0, int(rel_to_rhs), poll_every)
        st = SolveStats()
        rc = load_library().ell_mg_solve(self._h, _dev(f), _dev(u), ctypes.byref(o), ctypes.byref(st),
                                         _stream(stream))
        if check:
            _check(rc, allow=(ELL_OK, ELL_NOT_CONVERGED))
        return u, Stats(st.iters, st.status, st.r0_norm, st.r_norm, st.true_r_norm, st.b_norm)

    # ---- level entry points ----------------------------------------------------------
    def level_elems(self, level: int) -> int:
        return int(load_library().ell_level_elems(self._h, level))

    def level_layout(self, level: int):
        """(columns per colour H, plane stride S, colour stride C) of a level."""
        v = [ctypes.c_int64() for _ in range(3)]
        _check(load_library().ell_level_layout(self._h, level, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def level_empty(self, level: int) -> torch.Tensor:
        return torch.zeros(self.level_elems(level), dtype=self.elem_dtype, device="cuda")

    def to_split(self, level: int, src: torch.Tensor, dst: Optional[torch.Tensor] = None, stream=None):
        dst = self.level_empty(level) if dst is None else dst
        _check(load_library().ell_to_split(self._h, level, _dev(src), _dev(dst, self.elem_dtype),
                                           _stream(stream)))
        return dst

    def from_split(self, level: int, src: torch.Tensor, dst: torch.Tensor, stream=None):
        _check(load_library().ell_from_split(self._h, level, _dev(src, self.elem_dtype), _dev(dst),
                                             _stream(stream)))
        return dst

    def level_smooth(self, level, colour, b, u, zero_init=False, stream=None):
        _check(load_library().ell_level_smooth(self._h, level, colour, int(zero_init),
                                               _dev(b, self.elem_dtype), _dev(u, self.elem_dtype),
                                               _stream(stream)))
        return u

    def level_resid_restrict(self, level, b, u, bc, black_zero=False, stream=None):
        _check(load_library().ell_level_resid_restrict(
            self._h, level, _dev(b, self.elem_dtype), _dev(u, self.elem_dtype),
            _dev(bc, self.elem_dtype), int(black_zero), _stream(stream)))
        return bc

    def level_prolong_add(self, level, uc, u, red_only=False, stream=None):
        _check(load_library().ell_level_prolong_add(self._h, level, _dev(uc, self.elem_dtype),
                                                    _dev(u, self.elem_dtype), int(red_only),
                                                    _stream(stream)))
        return u

    def level_apply(self, level, x, y, stream=None):
        _check(load_library().ell_level_apply(self._h, level, _dev(x, self.elem_dtype),
                                              _dev(y, self.elem_dtype), _stream(stream)))
        return y

    # ---- measurement -------------------------------------------------------------------
    def profile_enable(self, family: int, max_events: int):
        _check(load_library().ell_profile_enable(self._h, family, max_events))

    def profile_pause(self, family: int, paused: bool = True):
        _check(load_library().ell_profile_pause(self._h, family, int(bool(paused))))

    def profile_read(self, family: int):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        _check(load_library().ell_profile_read(self._h, family, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def profile_times(self, family: int) -> np.ndarray:
        """Per-launch times (ms) of the recorded launches, in launch order."""
        n, _ = self.profile_read(family)
        buf = (ctypes.c_float * max(n, 1))()
        got = load_library().ell_profile_times(self._h, family, buf, n)
        _check(0 if got >= 0 else got)
        return np.frombuffer(buf, dtype=np.float32, count=n).astype(np.float64)


class BatchGrid(Grid):
    """A grid owned by a Batch (created with the batch's uniform layout)."""

    def __init__(self, batch: "Batch", nx, ny, nz, hx, hy, omega2, dz, lambda2, n_levels=0, nu_pre=1,
                 nu_post=1, nu_coarse=1, rho=1.0, prolong=0, precision="fp64"):
        L = load_library()
        d, keep = make_desc(nx, ny, nz, hx, hy, omega2, dz, lambda2, n_levels, nu_pre, nu_post,
                            nu_coarse, rho, prolong, precision)
        h = ctypes.c_void_p()
        _check(L.ell_batch_grid(batch._h, ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._batch = batch
        self.nx, self.ny, self.nz = nx, ny, nz
        self.precision = d.precision
        self.levels = L.ell_grid_levels(h)
        self.bytes = int(L.ell_grid_bytes(ctypes.byref(d)))

    def close(self):
        if getattr(self, "_h", None) and getattr(self._batch, "_h", None):
            load_library().ell_batch_release(self._batch._h, self._h)
        self._h = None


class Batch:
    """Grouped-launch batch engine with continuous admission (see ell.h)."""

    def __init__(self, hbm_budget_bytes: int):
        h = ctypes.c_void_p()
        _check(load_library().ell_batch_create(int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def grid(self, p=None, precision="fp64", **kw) -> BatchGrid:
        if p is not None:
            args = dict(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, omega2=p.omega2, dz=p.dz,
                        lambda2=p.lambda2, n_levels=p.n_levels, nu_pre=p.nu_pre,
                        nu_post=p.nu_post, nu_coarse=p.nu_coarse, rho=p.rho, prolong=p.prolong)
            args.update(kw)
            kw = args
        return BatchGrid(self, precision=precision, **kw)

    def bytes_in_use(self) -> int:
        return int(load_library().ell_batch_bytes_in_use(self._h))

    def submit(self, grids, fs, us, rtol=1e-5, atol=0.0, maxiter=500, flexible=True,
               rel_to_rhs=False, poll_every=4) -> int:
        n = len(grids)
        assert len(fs) == n and len(us) == n
        G = (ctypes.c_void_p * n)(*[g._h for g in grids])
        F = (ctypes.c_void_p * n)(*[_dev(f).value for f in fs])
        U = (ctypes.c_void_p * n)(*[_dev(u).value for u in us])
        o = SolveOpts(rtol, atol, maxiter, int(flexible), int(rel_to_rhs), poll_every)
        t = ctypes.c_uint64()
        # the engine reads the vectors on its own stream: make them ready first
        torch.cuda.current_stream().synchronize()
        _check(load_library().ell_batch_submit(self._h, n, G, F, U, ctypes.byref(o), ctypes.byref(t)))
        self._keep[t.value] = (fs, us, n)
        return t.value

    def _stats(self, buf, n):
        return [Stats(s.iters, s.status, s.r0_norm, s.r_norm, s.true_r_norm, s.b_norm) for s in buf[:n]]

    def poll(self, ticket: int):
        n = self._keep[ticket][2]
        buf = (SolveStats * n)()
        rc = load_library().ell_batch_poll(self._h, ticket, buf)
        if rc == ELL_PENDING:
            return None
        _check(rc, allow=(ELL_OK, ELL_NOT_CONVERGED))
        return self._stats(buf, n)

    def wait(self, ticket: int, check=True):
        n = self._keep[ticket][2]
        buf = (SolveStats * n)()
        rc = load_library().ell_batch_wait(self._h, ticket, buf)
        self._keep.pop(ticket, None)
        if check:
            _check(rc, allow=(ELL_OK, ELL_NOT_CONVERGED))
        return self._stats(buf, n)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ell_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
