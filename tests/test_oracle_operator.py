"""Pins of the oracle's operator (Sec. 3 eq. ModelEquation, Sec. 3.1 finite
volumes) against facts fixed by the mathematics, not by the oracle's code."""
import math

import numpy as np
import pytest

from helpers import closed_form_mu, dense_from_apply, mode, small_grid, volumes


@pytest.mark.parametrize("nx,ny,nz,hx,hy", [
    (4, 6, 5, 0.25, 1.0 / 6.0),
    (8, 8, 4, 1.0 / 8, 1.0 / 8),
    (2, 4, 3, 0.5, 0.3),
    (1, 6, 4, 1.0, 0.2),
    (6, 1, 4, 0.2, 1.0),
    (1, 1, 7, 1.0, 1.0),
])
def test_fourier_cosine_eigenmode(orc, nx, ny, nz, hx, hy):
    """Uniform dz, constant lambda^2: cos(2pi(pi/nx+qj/ny)) cos(pi m (k+1/2)/nz) is an
    eigenvector of the 7-point operator with A phi = V mu phi (discrete Fourier
    in the periodic directions, DCT-II for the Neumann column)."""
    g = small_grid(orc, nx, ny, nz, graded=False, hx=hx, hy=hy, omega2=0.37)
    V = volumes(g)
    for p in range(nx):
        for q in range(ny):
            for m in range(nz):
                for phase in (0.0, 0.7):
                    phi = mode(g, p, q, m, phase)
                    mu = closed_form_mu(g, p, q, m)
                    y = orc.apply(g, phi)
                    err = np.abs(y - V * mu * phi).max()
                    assert err <= 1e-13 * (V * mu).max(), (p, q, m, err)


def test_constants_give_volumes(orc):
    """The Laplacian parts annihilate constants, so A 1 = V exactly."""
    g = small_grid(orc, 8, 6, 9)
    y = orc.apply(g, np.ones(g.shape))
    np.testing.assert_array_equal(y, volumes(g))


@pytest.mark.parametrize("shape", [(4, 4, 6), (8, 2, 5), (2, 2, 3), (1, 4, 4), (6, 8, 12)])
def test_symmetric_positive(orc, shape):
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=nx * 31 + nz)
    rng = np.random.default_rng(3)
    V = volumes(g)
    for _ in range(5):
        u = rng.standard_normal(g.shape)
        v = rng.standard_normal(g.shape)
        uAv = float((u * orc.apply(g, v)).sum())
        vAu = float((v * orc.apply(g, u)).sum())
        scale = float(np.abs(u * orc.apply_abs(g, v)).sum())
        assert abs(uAv - vAu) <= 1e-14 * scale
        uAu = float((u * orc.apply(g, u)).sum())
        # the Laplacian parts are positive semi-definite: u'Au >= u'Vu > 0
        assert uAu >= float((V * u * u).sum()) * (1 - 1e-12) > 0


def test_dense_structure(orc):
    """Dense matrix on a 4x4x3 grid: 7-point pattern with periodic wrap,
    non-positive off-diagonals, rows summing to the cell volume, symmetric."""
    g = small_grid(orc, 4, 4, 3)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    n = A.shape[0]
    assert np.allclose(A, A.T, rtol=1e-14, atol=0)
    idx = lambda i, j, k: (k * g.ny + j) * g.nx + i
    V = volumes(g).ravel()
    for k in range(g.nz):
        for j in range(g.ny):
            for i in range(g.nx):
                c = idx(i, j, k)
                allowed = {c, idx((i - 1) % 4, j, k), idx((i + 1) % 4, j, k),
                           idx(i, (j - 1) % 4, k), idx(i, (j + 1) % 4, k)}
                if k > 0:
                    allowed.add(idx(i, j, k - 1))
                if k < g.nz - 1:
                    allowed.add(idx(i, j, k + 1))
                nz_cols = set(np.nonzero(A[c])[0].tolist())
                assert nz_cols == allowed
                off = [A[c, d] for d in nz_cols if d != c]
                assert all(o < 0 for o in off)
                assert math.isclose(A[c].sum(), V[c], rel_tol=1e-10, abs_tol=1e-12 * A[c, c])
    assert np.all(np.linalg.eigvalsh(A) > 0)
    assert n == 48


def test_vertical_face_constant_flux(orc):
    """Graded dz and variable lambda^2 in one column: a profile that is linear
    inside each cell with the same flux F = -lambda^2 du/dz everywhere (which
    solves d/dz(lambda^2 du/dz) = 0 exactly) has cell-centre differences
    u_{k+1} - u_k = -F (dz_k/(2 lam_k) + dz_{k+1}/(2 lam_{k+1})).  The finite-volume
    flux balance of such a profile vanishes in the interior, and at the two
    Neumann ends it equals the boundary flux omega^2 hx hy F."""
    nz = 9
    rng = np.random.default_rng(11)
    dz = rng.uniform(0.2, 3.0, nz) * 1e-3
    lam = np.exp(rng.uniform(-3, 3, nz))
    g = orc.Grid(1, 1, nz, 0.3, 0.2, 0.05, dz, lam)
    F = 0.8
    u = np.zeros(nz)
    u[0] = 1.3
    for k in range(nz - 1):
        # exact integral of du/dz = -F/lambda^2 from centre k to centre k+1
        u[k + 1] = u[k] - F * (0.5 * dz[k] / lam[k] + 0.5 * dz[k + 1] / lam[k + 1])
    y = orc.apply(g, u.reshape(nz, 1, 1)).ravel()
    V = g.hx * g.hy * dz
    flux = g.omega2 * g.hx * g.hy * F
    expect = V * u
    expect[0] += flux          # cell 0 loses F through its top face only
    expect[-1] -= flux         # cell nz-1 gains F through its bottom face only
    scale = V * np.abs(u) + flux
    assert np.all(np.abs(y - expect) <= 1e-12 * scale)


def test_coarse_levels_rediscretised(orc):
    """Every level uses the same finite-volume formula on h_l = 2^l h, so the
    closed-form eigenvalue holds on the coarse geometry with doubled spacing."""
    g = small_grid(orc, 8, 8, 4, graded=False, omega2=0.2)
    c = g.coarse()
    assert (c.nx, c.ny, c.hx, c.hy) == (4, 4, 2 * g.hx, 2 * g.hy)
    V = volumes(c)
    for (p, q, m) in [(1, 0, 0), (1, 2, 3), (3, 3, 1)]:
        phi = mode(c, p, q, m)
        y = orc.apply(c, phi)
        assert np.abs(y - V * closed_form_mu(c, p, q, m) * phi).max() < 1e-12 * V.max() * 1e3


def test_standard_depth(orc):
    assert orc.standard_levels(32, 32) == 6      # 32..1
    assert orc.standard_levels(512, 512) == 10
    assert orc.standard_levels(96, 96) == 5      # 96, 48, 24, 12, 6
    assert orc.standard_levels(192, 192) == 6
    assert orc.standard_levels(4, 2) == 2        # 4x2 -> 2x1
    assert orc.standard_levels(6, 6) == 1
    assert orc.standard_levels(1, 1) == 1


@pytest.mark.parametrize("shape", [(4, 4, 4), (2, 4, 3), (4, 2, 4), (1, 4, 3), (4, 1, 3), (1, 1, 4), (2, 2, 2)])
def test_apply_abs_is_abs_matrix_times_abs_vector(orc, shape):
    """The error scale of the operator comparisons, sum over the terms of
    (A x)_c of their absolute values, is |A| |x| of the dense matrix (every
    coefficient is positive, so |V x_c| + sum T (|x_c| + |x_nbr|) equals the
    absolute diagonal times |x_c| plus the absolute off-diagonals times the
    neighbours).  The dense matrix comes from the operator, which the closed
    forms above pin; periodic neighbours that coincide (size 2) and omitted
    faces (size 1) are covered."""
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=5 * nx + 3 * ny + nz)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    rng = np.random.default_rng(17)
    for _ in range(4):
        x = rng.standard_normal(g.shape)
        got = orc.apply_abs(g, x).ravel()
        ref = np.abs(A) @ np.abs(x.ravel())
        assert np.all(np.abs(got - ref) <= 1e-13 * ref), np.abs(got - ref).max()
        # and it bounds the operator itself
        assert np.all(np.abs(orc.apply(g, x)).ravel() <= got * (1 + 1e-14))
