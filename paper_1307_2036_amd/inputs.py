"""Seeded synthetic inputs for the anisotropic pressure-correction problem.

This module only *draws* inputs: vertical spacings, the vertical coefficient
profile lambda^2(z), right-hand sides and the workload descriptions.  It holds
none of the solver's arithmetic (no operator, smoother, transfer or Krylov
step), so both the FP64 reference implementation under ``oracle/`` and the HIP
library receive exactly the same bytes from here.

Shapes follow the paper's weak-scaling runs (n_x^2 x 128 columns, Sec. 7.1 and
Table 1); the right-hand side, which the paper never states, is a seeded random
field with its volume-weighted mean removed.

Arrays use the plane-major layout idx = (k*ny + j)*nx + i, i.e. numpy shape
(nz, ny, nx).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

DEFAULT_SEED_BASE = 1307


def seed_for(config: int, instance: int = 0, stream: int = 0) -> int:
    """Default seed: 1307 + 100*config + instance (+ 100000*stream)."""
    return DEFAULT_SEED_BASE + 100 * config + instance + 100000 * stream


# --------------------------------------------------------------------------
# vertical grids
# --------------------------------------------------------------------------
def dz_uniform(nz: int, depth: float) -> np.ndarray:
    return np.full(nz, depth / nz, dtype=np.float64)


def dz_quadratic(nz: int, depth: float = 1.0 / 50.0) -> np.ndarray:
    """Thicknesses growing like (k+1)^2, normalised to the total depth."""
    w = (np.arange(nz, dtype=np.float64) + 1.0) ** 2
    return depth * w / w.sum()


def dz_paper_grading(nz: int, depth: float = 0.01) -> np.ndarray:
    """The paper's level placement r_k = 1 + H (k/nz)^2 (eq. VerticalGrading):
    thicknesses H((k+1)^2 - k^2)/nz^2, i.e. growing linearly with height."""
    k = np.arange(nz + 1, dtype=np.float64)
    r = depth * (k / nz) ** 2
    return np.diff(r)


def lambda2_perturbed(h: float, dz: np.ndarray, sigma: float, seed: int,
                      n_modes: int = 8) -> np.ndarray:
    """lambda^2_k = (h/dz_k)^2 * exp(sigma * g_k).

    g is a smooth random profile in height: sum_{m=1..n_modes} xi_m cos(pi m zeta_k)
    with xi_m ~ N(0,1) from ``seed`` and zeta_k the cell-centre height divided by
    the depth, rescaled to unit RMS over k.  sigma = 0 gives the unperturbed
    (h/dz)^2 profile.
    """
    dz = np.asarray(dz, dtype=np.float64)
    depth = dz.sum()
    zc = (np.cumsum(dz) - 0.5 * dz) / depth
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(n_modes)
    g = np.zeros_like(zc)
    for m in range(1, n_modes + 1):
        g += xi[m - 1] * np.cos(math.pi * m * zc)
    rms = math.sqrt(float(np.mean(g * g)))
    if rms > 0:
        g = g / rms
    return (h / dz) ** 2 * np.exp(sigma * g)


def lambda2_3d(nx: int, ny: int, lam_z: np.ndarray, sigma_h: float, seed: int,
               n_modes: int = 3) -> np.ndarray:
    """A 3D cell field lambda^2(i,j,k) = lambda^2_k * exp(sigma_h * g_k(x, y)),
    shape (nz, ny, nx): the column profile lam_z modulated horizontally by a
    smooth periodic random field whose pattern changes with height,
    g = sum over 0 <= p, q <= n_modes, (p, q) != (0, 0), of
    (xi_pq + eta_pq zeta_k) cos(2 pi (p x + q y) + phi_pq), x = (i+1/2)/nx,
    y = (j+1/2)/ny, zeta_k = (k+1/2)/nz, xi, eta ~ N(0,1), phi ~ U[0, 2 pi),
    rescaled to unit RMS.  It stands in for the horizontally varying metric
    terms of the paper's cubed-sphere panel, which make every column's
    vertical coefficients different (Sec. 3, Sec. 6.2.1)."""
    lam_z = np.asarray(lam_z, dtype=np.float64)
    nz = len(lam_z)
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    zeta = (np.arange(nz) + 0.5) / nz
    g = np.zeros((nz, ny, nx))
    for p in range(n_modes + 1):
        for q in range(n_modes + 1):
            if p == 0 and q == 0:
                continue
            xi, eta = rng.standard_normal(2)
            phi = rng.uniform(0.0, 2.0 * math.pi)
            wave = np.cos(2.0 * math.pi * (p * x[None, :] + q * y[:, None]) + phi)
            g += (xi + eta * zeta)[:, None, None] * wave[None, :, :]
    rms = math.sqrt(float(np.mean(g * g)))
    if rms > 0:
        g = g / rms
    return np.ascontiguousarray(lam_z[:, None, None] * np.exp(sigma_h * g))


# --------------------------------------------------------------------------
# right-hand sides
# --------------------------------------------------------------------------
def _remove_volume_mean(f: np.ndarray, dz: np.ndarray) -> np.ndarray:
    # cell volumes are hx*hy*dz_k; the horizontal factor cancels in the mean
    w = np.asarray(dz, dtype=np.float64)[:, None, None]
    mean = float((f * w).sum() / (w.sum() * f.shape[1] * f.shape[2]))
    return f - mean


def rhs_uniform(nx: int, ny: int, dz: np.ndarray, seed: int) -> np.ndarray:
    """f ~ U[-1, 1] i.i.d., volume-weighted mean removed; shape (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, size=(len(dz), ny, nx))
    return np.ascontiguousarray(_remove_volume_mean(f, dz))


def rhs_normal(nx: int, ny: int, dz: np.ndarray, seed: int) -> np.ndarray:
    """f ~ N(0, 1) i.i.d., volume-weighted mean removed; shape (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(size=(len(dz), ny, nx))
    return np.ascontiguousarray(_remove_volume_mean(f, dz))


def random_field(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(nz, ny, nx))


# --------------------------------------------------------------------------
# paper parameters (Sec. 3, eq. omega2lambda2 and Table 1)
# --------------------------------------------------------------------------
EARTH_RADIUS_M = 6.371e6
C_H = 550.0          # fastest wave speed [m/s]
N_BG = 0.018         # buoyancy frequency [1/s]
ALPHA = 0.5          # off-centering parameter


def paper_omega2(dt: float) -> float:
    return (ALPHA * C_H * dt / EARTH_RADIUS_M) ** 2


def paper_lambda2(dt: float) -> float:
    return 1.0 / (1.0 + (ALPHA * dt * N_BG) ** 2)


def paper_dx_m(nx: int) -> float:
    """Typical horizontal spacing of the cubed-sphere panel, 2 pi R / (4 nx)."""
    return 2.0 * math.pi * EARTH_RADIUS_M / (4.0 * nx)


# --------------------------------------------------------------------------
# workload descriptions
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """One solve: grid, coefficients, right-hand side and multigrid options."""
    name: str
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    dz: np.ndarray
    lambda2: np.ndarray
    omega2: float
    f: Optional[np.ndarray] = None
    n_levels: int = 0          # 0 = standard depth
    nu_pre: int = 1
    nu_post: int = 1
    nu_coarse: int = 1
    rho: float = 1.0
    prolong: int = 0           # 0 bilinear, 1 piecewise constant
    rtol: float = 1e-5
    seeds: dict = field(default_factory=dict)
    # None, or a 3D cell field lambda^2 of shape (nz, ny, nx) that replaces
    # lambda2 (horizontally varying vertical coefficients)
    lambda2_3d: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def config0(seed: Optional[int] = None) -> Problem:
    """32x32x16, h=1/32, dz=1/16 uniform, omega^2=1e-2, lambda^2=1e4, f~U[-1,1]."""
    seed = seed_for(0) if seed is None else seed
    nx = ny = 32
    nz = 16
    dz = dz_uniform(nz, 1.0)
    lam = np.full(nz, 1e4)
    f = rhs_uniform(nx, ny, dz, seed)
    return Problem("config0_32x32x16_fp64", nx, ny, nz, 1.0 / nx, 1.0 / ny, dz, lam,
                   1e-2, f, n_levels=0, nu_coarse=1, seeds={"f": seed})


def graded_problem(name: str, nx: int, nz: int, omega2: float, seed_f: int,
                   seed_lambda: int, n_levels: int = 0, nu_coarse: int = 1,
                   with_f: bool = True, sigma: float = 0.3,
                   depth: float = 1.0 / 50.0) -> Problem:
    """Production-shaped problem: nx^2 x nz, h = 1/nx, dz ~ (k+1)^2 over depth 1/50,
    lambda^2 = (h/dz)^2 * smooth log-normal perturbation, f ~ N(0,1)."""
    h = 1.0 / nx
    dz = dz_quadratic(nz, depth)
    lam = lambda2_perturbed(h, dz, sigma, seed_lambda)
    f = rhs_normal(nx, nx, dz, seed_f) if with_f else None
    return Problem(name, nx, nx, nz, h, h, dz, lam, omega2, f, n_levels=n_levels,
                   nu_coarse=nu_coarse, seeds={"f": seed_f, "lambda": seed_lambda})


def paper_graded_problem(name: str, nx: int, ny: int, nz: int, omega2: float, seed_f: int,
                         seed_lambda: int, depth: float = 1.0, sigma: float = 0.3) -> Problem:
    """nx x ny x nz with the paper's level placement (eq. VerticalGrading,
    thicknesses growing linearly with height), h = 1/nx and 1/ny,
    lambda^2 = (hx/dz)^2 * smooth log-normal perturbation, f ~ N(0,1).  Over
    depth 1 the vertical couplings stay within ~1e15 of the cell volumes, so
    FP64 resolves the residual of the solve (the quadratic grading over depth
    1/50 does not at 192 or more levels)."""
    dz = dz_paper_grading(nz, depth)
    lam = lambda2_perturbed(1.0 / nx, dz, sigma, seed_lambda)
    f = rhs_normal(nx, ny, dz, seed_f)
    return Problem(name, nx, ny, nz, 1.0 / nx, 1.0 / ny, dz, lam, omega2, f,
                   seeds={"f": seed_f, "lambda": seed_lambda})


def varying_problem(nx: int = 512, nz: int = 128, n_levels: int = 4, nu_coarse: int = 5,
                    sigma_h: float = 0.5, with_f: bool = True) -> Problem:
    """The 512 x 512 x 128 graded problem (four levels, five coarse sweeps) with its lambda^2 profile
    modulated horizontally (lambda2_3d, sigma_h = 0.5): every column has its own
    vertical coefficients."""
    p = graded_problem(f"varying_{nx}x{nx}x{nz}_L{n_levels}", nx, nz, 1e-2, seed_for(5),
                       seed_for(5, stream=1), n_levels=n_levels, nu_coarse=nu_coarse,
                       with_f=with_f)
    p.lambda2_3d = lambda2_3d(nx, nx, p.lambda2, sigma_h, seed_for(5, stream=2))
    p.seeds["lambda2_3d"] = seed_for(5, stream=2)
    return p


def config1(n_levels: int = 4, nu_coarse: int = 5, nx: int = 512, nz: int = 128,
            with_f: bool = True) -> Problem:
    """512x512x128 graded, omega^2 = 1e-2, four-level hierarchy, 5 coarse sweeps."""
    return graded_problem(f"config1_{nx}x{nx}x{nz}_L{n_levels}", nx, nz, 1e-2,
                          seed_for(1), seed_for(1, stream=1), n_levels=n_levels,
                          nu_coarse=nu_coarse, with_f=with_f)


def config2(omega2: float = 1e-2, nx: int = 1024, nz: int = 128,
            with_f: bool = True) -> Problem:
    """1024x1024x128 graded, omega^2 in {1e-3, 1e-2, 1e-1}, standard depth."""
    return graded_problem(f"config2_{nx}x{nx}x{nz}_w{omega2:g}", nx, nz, omega2,
                          seed_for(2), seed_for(2, stream=1), with_f=with_f)


def config3_instances(count: int = 64, seed: Optional[int] = None,
                      with_f: bool = True):
    """Uneven batch: nx in {64,96,128,192,256}, nz in {64,96,128},
    log-uniform omega^2 in [1e-3, 1e-1]."""
    seed = seed_for(3) if seed is None else seed
    rng = np.random.default_rng(seed)
    out = []
    for idx in range(count):
        nx = int(rng.choice([64, 96, 128, 192, 256]))
        nz = int(rng.choice([64, 96, 128]))
        omega2 = float(10.0 ** rng.uniform(-3.0, -1.0))
        out.append(graded_problem(f"config3_{idx}_{nx}x{nx}x{nz}", nx, nz, omega2,
                                  seed_for(3, idx), seed_for(3, idx, stream=1),
                                  with_f=with_f))
    return out
