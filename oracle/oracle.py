"""ctypes wrapper of the FP64 reference implementation in ``ell_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The HIP library never
imports this module and this module never imports the HIP library.

All arrays are float64 numpy arrays in plane-major layout, shape (nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ell_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


class Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("omega2", ctypes.c_double), ("dz", _dp), ("lambda2", _dp), ("tz3", _dp)]


class MG(ctypes.Structure):
    _fields_ = [("g", Geom), ("n_levels", ctypes.c_int), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("nu_coarse", ctypes.c_int),
                ("rho", ctypes.c_double), ("prolong", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("flexible", ctypes.c_int),
                ("rel_to_rhs", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("r0_norm", ctypes.c_double),
                ("r_norm", ctypes.c_double), ("true_r_norm", ctypes.c_double),
                ("b_norm", ctypes.c_double), ("status", ctypes.c_int)]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        L.orc_apply.argtypes = [ctypes.POINTER(Geom), _dp, _dp]
        L.orc_apply_abs.argtypes = [ctypes.POINTER(Geom), _dp, _dp]
        L.orc_smooth_colour.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_residual.argtypes = [ctypes.POINTER(Geom), _dp, _dp, _dp]
        L.orc_restrict.argtypes = [ctypes.POINTER(Geom), _dp, _dp]
        L.orc_prolong_add.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, _dp, _dp]
        L.orc_vcycle.argtypes = [ctypes.POINTER(MG), _dp, _dp]
        L.orc_vcycle.restype = ctypes.c_int
        L.orc_pcg.argtypes = [ctypes.POINTER(MG), ctypes.POINTER(Opts), _dp, _dp, ctypes.POINTER(Stats)]
        L.orc_pcg.restype = ctypes.c_int
        L.orc_mg_solve.argtypes = [ctypes.POINTER(MG), ctypes.POINTER(Opts), _dp, _dp, ctypes.POINTER(Stats)]
        L.orc_mg_solve.restype = ctypes.c_int
        L.orc_num_levels.argtypes = [ctypes.POINTER(MG)]
        L.orc_num_levels.restype = ctypes.c_int
        L.orc_standard_levels.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_standard_levels.restype = ctypes.c_int
        L.orc_level_coeffs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_thomas_plain.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_column_solve.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_tz3_from_lambda2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        L.orc_tz3_coarsen.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Grid:
    """Finest-level geometry plus multigrid options."""
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    omega2: float
    dz: np.ndarray
    lambda2: np.ndarray
    n_levels: int = 0
    nu_pre: int = 1
    nu_post: int = 1
    nu_coarse: int = 1
    rho: float = 1.0
    prolong: int = 0
    # None: vertical faces from lambda2(z); else the per-column vertical face
    # coefficients, shape (nz+1, ny, nx) (see tz3_from_lambda2)
    tz3: Optional[np.ndarray] = None

    def __post_init__(self):
        self.dz = _c(self.dz)
        self.lambda2 = _c(self.lambda2)
        assert self.dz.shape == (self.nz,) and self.lambda2.shape == (self.nz,)
        if self.tz3 is not None:
            self.tz3 = _c(self.tz3)
            assert self.tz3.shape == (self.nz + 1, self.ny, self.nx)

    @classmethod
    def from_problem(cls, p, **over):
        kw = dict(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, omega2=p.omega2, dz=p.dz,
                  lambda2=p.lambda2, n_levels=p.n_levels, nu_pre=p.nu_pre, nu_post=p.nu_post,
                  nu_coarse=p.nu_coarse, rho=p.rho, prolong=p.prolong)
        lam3 = getattr(p, "lambda2_3d", None)
        if lam3 is not None:
            kw["tz3"] = tz3_from_lambda2(p.nx, p.ny, p.nz, p.hx, p.hy, p.omega2, p.dz, lam3)
        kw.update(over)
        return cls(**kw)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def geom(self) -> Geom:
        return Geom(self.nx, self.ny, self.nz, self.hx, self.hy, self.omega2,
                    _ptr(self.dz), _ptr(self.lambda2),
                    None if self.tz3 is None else _ptr(self.tz3))

    def mg(self) -> MG:
        return MG(self.geom(), self.n_levels, self.nu_pre, self.nu_post, self.nu_coarse,
                  self.rho, self.prolong)

    def coarse(self) -> "Grid":
        return Grid(self.nx // 2, self.ny // 2, self.nz, 2 * self.hx, 2 * self.hy, self.omega2,
                    self.dz, self.lambda2, 0, self.nu_pre, self.nu_post, self.nu_coarse,
                    self.rho, self.prolong,
                    None if self.tz3 is None else tz3_coarsen(self.tz3))


def tz3_from_lambda2(nx, ny, nz, hx, hy, omega2, dz, lambda2_3d) -> np.ndarray:
    """Per-column vertical face coefficients, shape (nz+1, ny, nx), of a 3D
    cell field lambda^2 of shape (nz, ny, nx)."""
    dz = _c(dz)
    lam = _c(lambda2_3d).reshape(nz, ny, nx)
    out = np.empty((nz + 1, ny, nx))
    lib().orc_tz3_from_lambda2(nx, ny, nz, hx, hy, omega2, _ptr(dz), _ptr(lam), _ptr(out))
    return out


def tz3_coarsen(tz3) -> np.ndarray:
    """Faces of the next coarser level: each coarse face is the sum of its
    four children's."""
    tz3 = _c(tz3)
    nz1, ny, nx = tz3.shape
    out = np.empty((nz1, ny // 2, nx // 2))
    lib().orc_tz3_coarsen(nx, ny, nz1 - 1, _ptr(tz3), _ptr(out))
    return out


def level_coeffs(g: Grid):
    """(V, Tx, Ty, Tz[nz+1], s) of the grid's finest level."""
    nz = g.nz
    V, Tx, Ty, s = (np.zeros(nz) for _ in range(4))
    Tz = np.zeros(nz + 1)
    lib().orc_level_coeffs(g.nx, g.ny, nz, g.hx, g.hy, g.omega2, _ptr(g.dz), _ptr(g.lambda2),
                           _ptr(V), _ptr(Tx), _ptr(Ty), _ptr(Tz), _ptr(s))
    return V, Tx, Ty, Tz, s


def apply(g: Grid, x) -> np.ndarray:
    x = _c(x).reshape(g.shape)
    y = np.empty_like(x)
    gg = g.geom()
    lib().orc_apply(ctypes.byref(gg), _ptr(x), _ptr(y))
    return y


def apply_abs(g: Grid, x) -> np.ndarray:
    x = _c(x).reshape(g.shape)
    y = np.empty_like(x)
    gg = g.geom()
    lib().orc_apply_abs(ctypes.byref(gg), _ptr(x), _ptr(y))
    return y


def smooth_colour(g: Grid, colour: int, b, u, rho: float = 1.0) -> np.ndarray:
    b = _c(b).reshape(g.shape)
    u = _c(u).reshape(g.shape).copy()
    gg = g.geom()
    lib().orc_smooth_colour(ctypes.byref(gg), colour, rho, _ptr(b), _ptr(u))
    return u


def residual(g: Grid, b, u) -> np.ndarray:
    b = _c(b).reshape(g.shape)
    u = _c(u).reshape(g.shape)
    r = np.empty_like(b)
    gg = g.geom()
    lib().orc_residual(ctypes.byref(gg), _ptr(b), _ptr(u), _ptr(r))
    return r


def restrict(g: Grid, r) -> np.ndarray:
    r = _c(r).reshape(g.shape)
    bc = np.empty((g.nz, g.ny // 2, g.nx // 2))
    gg = g.geom()
    lib().orc_restrict(ctypes.byref(gg), _ptr(r), _ptr(bc))
    return bc


def prolong_add(g: Grid, uc, u, mode: int = 0) -> np.ndarray:
    uc = _c(uc).reshape(g.nz, g.ny // 2, g.nx // 2)
    u = _c(u).reshape(g.shape).copy()
    gg = g.geom()
    lib().orc_prolong_add(ctypes.byref(gg), mode, _ptr(uc), _ptr(u))
    return u


def num_levels(g: Grid) -> int:
    m = g.mg()
    return lib().orc_num_levels(ctypes.byref(m))


def standard_levels(nx: int, ny: int) -> int:
    return lib().orc_standard_levels(nx, ny)


def vcycle(g: Grid, r) -> np.ndarray:
    r = _c(r).reshape(g.shape)
    z = np.empty_like(r)
    m = g.mg()
    rc = lib().orc_vcycle(ctypes.byref(m), _ptr(r), _ptr(z))
    if rc != 0:
        raise ValueError("invalid multigrid hierarchy")
    return z


def pcg(g: Grid, f, u0=None, rtol: float = 1e-5, atol: float = 0.0, maxiter: int = 500,
        flexible: bool = True, rel_to_rhs: bool = False):
    """Solve A u = V f; returns (u, stats dict)."""
    f = _c(f).reshape(g.shape)
    u = np.zeros(g.shape) if u0 is None else _c(u0).reshape(g.shape).copy()
    m = g.mg()
    o = Opts(rtol, atol, maxiter, int(flexible), int(rel_to_rhs))
    st = Stats()
    rc = lib().orc_pcg(ctypes.byref(m), ctypes.byref(o), _ptr(f), _ptr(u), ctypes.byref(st))
    if rc != 0:
        raise ValueError("invalid multigrid hierarchy")
    return u, dict(iters=st.iters, r0_norm=st.r0_norm, r_norm=st.r_norm,
                   true_r_norm=st.true_r_norm, b_norm=st.b_norm, status=st.status)


def mg_solve(g: Grid, f, u0=None, rtol: float = 1e-5, atol: float = 0.0, maxiter: int = 500,
             rel_to_rhs: bool = False):
    """Stand-alone multigrid for A u = V f (repeated V-cycles); returns (u, stats dict)."""
    f = _c(f).reshape(g.shape)
    u = np.zeros(g.shape) if u0 is None else _c(u0).reshape(g.shape).copy()
    m = g.mg()
    o = Opts(rtol, atol, maxiter, 1, int(rel_to_rhs))
    st = Stats()
    rc = lib().orc_mg_solve(ctypes.byref(m), ctypes.byref(o), _ptr(f), _ptr(u), ctypes.byref(st))
    if rc != 0:
        raise ValueError("invalid multigrid hierarchy")
    return u, dict(iters=st.iters, r0_norm=st.r0_norm, r_norm=st.r_norm,
                   true_r_norm=st.true_r_norm, b_norm=st.b_norm, status=st.status)


def thomas_plain(a, b, c, f) -> np.ndarray:
    a, b, c, f = (_c(x) for x in (a, b, c, f))
    u = np.empty_like(f)
    lib().orc_thomas_plain(len(a), _ptr(a), _ptr(b), _ptr(c), _ptr(f), _ptr(u))
    return u


def column_solve(s, Tz, g) -> np.ndarray:
    s, Tz, g = (_c(x) for x in (s, Tz, g))
    nz = len(s)
    assert Tz.shape == (nz + 1,)
    w = np.empty(nz)
    work = np.empty(2 * nz)
    lib().orc_column_solve(nz, _ptr(s), _ptr(Tz), _ptr(g), _ptr(w), _ptr(work))
    return w


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(n)
