"""Shared test helpers: dense assembly through the oracle, small random grids,
index permutations for the colour-split device layout."""
from __future__ import annotations

import math

import numpy as np

from paper_1307_2036_amd import inputs as I


def dense_from_apply(apply, shape):
    """Dense matrix of a linear map given as a function on arrays of ``shape``."""
    n = int(np.prod(shape))
    M = np.empty((n, n))
    e = np.zeros(n)
    for c in range(n):
        e[c] = 1.0
        M[:, c] = apply(e.reshape(shape)).ravel()
        e[c] = 0.0
    return M


def small_grid(O, nx, ny, nz, graded=True, seed=7, omega2=None, hx=None, hy=None, **mg):
    """A small grid with graded spacing and a perturbed lambda^2 profile."""
    rng = np.random.default_rng(seed)
    hx = 1.0 / nx if hx is None else hx
    hy = 1.0 / ny if hy is None else hy
    if graded:
        dz = I.dz_quadratic(nz, 1.0 / 50.0)
        lam = I.lambda2_perturbed(hx, dz, 0.3, seed) * 1e-6
    else:
        dz = I.dz_uniform(nz, 1.0)
        lam = np.full(nz, 3.0)
    if omega2 is None:
        omega2 = float(10 ** rng.uniform(-3, -1))
    return O.Grid(nx, ny, nz, hx, hy, omega2, dz, lam, **mg)


def colour_columns(nx, ny, colour):
    return [(i, j) for j in range(ny) for i in range(nx) if (i + j) % 2 == colour]


def closed_form_mu(g, p, q, m):
    """Eigenvalue ratio of the Fourier x cosine mode for uniform dz and constant lambda^2."""
    dz = g.dz[0]
    lam = g.lambda2[0]
    t = 0.0
    if g.nx > 1:
        t += 4.0 / g.hx ** 2 * math.sin(math.pi * p / g.nx) ** 2
    if g.ny > 1:
        t += 4.0 / g.hy ** 2 * math.sin(math.pi * q / g.ny) ** 2
    t += lam * 4.0 / dz ** 2 * math.sin(math.pi * m / (2 * g.nz)) ** 2
    return 1.0 + g.omega2 * t


def mode(g, p, q, m, phase=0.0):
    k = np.arange(g.nz)[:, None, None]
    j = np.arange(g.ny)[None, :, None]
    i = np.arange(g.nx)[None, None, :]
    return (np.cos(2 * math.pi * (p * i / g.nx + q * j / g.ny) + phase)
            * np.cos(math.pi * m * (k + 0.5) / g.nz))


def volumes(g):
    return (g.hx * g.hy * g.dz)[:, None, None] * np.ones((1, g.ny, g.nx))
