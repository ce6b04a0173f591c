"""Pins of the oracle's horizontally varying vertical coefficients (a 3D
lambda^2 field, every column with its own vertical faces; the paper's model
equation, Sec. 3 eq. ModelEquation, with lambda^2 depending on all three
coordinates, discretised by the finite volumes of Sec. 3.1).

What fixes the results without the oracle's code:
  * a horizontally constant field is the z-only problem, which the other
    oracle pins already fix: every operation must agree bitwise, also on
    the coarse levels (summing four equal faces in pairs is exact);
  * the harmonic face rule is exact for piecewise constant lambda^2: the
    cell-centre samples of the continuum solution with constant vertical
    flux have that flux through every discrete face;
  * coarse faces are the sums of the children's: with piecewise constant
    prolongation P and sum restriction R, R A P is the coarse operator
    (Galerkin identity) on a 2 x 2 -> 1 x 1 hierarchy;
  * a column smoother sweep on a one-column grid is the exact solve, and
    CG converges to the dense solution;
  * A is symmetric positive definite; the V-cycle with piecewise constant
    prolongation and reversed colours is symmetric positive definite.
"""
import numpy as np
import pytest

from helpers import dense_from_apply, small_grid
from paper_1307_2036_amd import inputs as I
from test_oracle_vcycle import dense_R, dense_vcycle


def grid3(orc, nx, ny, nz, seed=3, sigma=0.8, graded=False, **kw):
    """A small grid with a 3D lambda^2 field: uniform levels (dense solves stay
    well conditioned) unless graded."""
    g = small_grid(orc, nx, ny, nz, graded=graded, seed=seed, **kw)
    lam3 = I.lambda2_3d(nx, ny, g.lambda2, sigma, seed + 11)
    g.tz3 = orc.tz3_from_lambda2(nx, ny, nz, g.hx, g.hy, g.omega2, g.dz, lam3)
    return g, lam3


def with_tz3(orc, g):
    """The same grid with its z-only faces given as per-column faces."""
    lam3 = np.broadcast_to(g.lambda2[:, None, None], g.shape).copy()
    g3 = orc.Grid(g.nx, g.ny, g.nz, g.hx, g.hy, g.omega2, g.dz, g.lambda2, g.n_levels, g.nu_pre,
                  g.nu_post, g.nu_coarse, g.rho, g.prolong,
                  orc.tz3_from_lambda2(g.nx, g.ny, g.nz, g.hx, g.hy, g.omega2, g.dz, lam3))
    return g3


@pytest.mark.parametrize("shape,levels", [((16, 8, 12), 3), ((8, 8, 5), 0), ((1, 8, 6), 0), ((8, 1, 6), 0)])
def test_horizontally_constant_field_is_the_z_only_problem(orc, shape, levels):
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=nx + nz, n_levels=levels)
    g3 = with_tz3(orc, g)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(g.shape)
    np.testing.assert_array_equal(orc.apply(g3, x), orc.apply(g, x))
    b = rng.standard_normal(g.shape)
    for c in (0, 1):
        np.testing.assert_array_equal(orc.smooth_colour(g3, c, b, x), orc.smooth_colour(g, c, b, x))
    np.testing.assert_array_equal(orc.vcycle(g3, b), orc.vcycle(g, b))
    f = rng.standard_normal(g.shape)
    u3, s3 = orc.pcg(g3, f, rtol=1e-8)
    u1, s1 = orc.pcg(g, f, rtol=1e-8)
    assert s3["iters"] == s1["iters"]
    np.testing.assert_array_equal(u3, u1)
    # coarse faces: four equal faces added in pairs give exactly the
    # re-discretised face of the coarse level
    gc, g3c = g.coarse(), g3.coarse()
    if nx > 1 and ny > 1:
        np.testing.assert_array_equal(orc.apply(g3c, x[:, ::2, ::2]), orc.apply(gc, x[:, ::2, ::2]))


def test_harmonic_faces_carry_a_constant_flux_exactly(orc):
    """One column, piecewise constant lambda^2 (four decades): integrate the
    continuum flux equation -omega^2 hx hy lambda^2 du/dz = F across each
    half cell and sample u at the cell centres; the vertical part of A u then
    vanishes in interior cells and is +F / -F in the bottom / top cell."""
    nz = 9
    rng = np.random.default_rng(2)
    dz = rng.uniform(0.5, 2.0, nz) * 0.1
    lam = 10.0 ** rng.uniform(-2, 2, nz)
    hx, hy, omega2, F = 0.3, 0.7, 0.05, 1.7
    u = np.zeros(nz)
    for k in range(nz - 1):
        # du/dz = -F / (omega^2 hx hy lambda^2) in each half cell
        u[k + 1] = u[k] - F / (omega2 * hx * hy) * (0.5 * dz[k] / lam[k] + 0.5 * dz[k + 1] / lam[k + 1])
    tz3 = orc.tz3_from_lambda2(1, 1, nz, hx, hy, omega2, dz, lam.reshape(nz, 1, 1))
    g = orc.Grid(1, 1, nz, hx, hy, omega2, dz, np.ones(nz), tz3=tz3)
    vert = orc.apply(g, u.reshape(nz, 1, 1)).ravel() - hx * hy * dz * u
    expect = np.zeros(nz)
    expect[0], expect[-1] = F, -F
    scale = np.abs(u).max() * tz3.max()
    assert np.abs(vert - expect).max() <= 1e-13 * scale


@pytest.mark.parametrize("nz", [1, 3, 6])
def test_coarse_faces_give_the_galerkin_operator(orc, nz):
    """2 x 2 x nz -> 1 x 1 x nz with piecewise constant prolongation: the
    horizontal differences of P e vanish, so R A P = 4 V_fine + summed
    vertical faces, which must be the coarse level's operator."""
    g, _ = grid3(orc, 2, 2, nz, seed=nz, graded=True)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    R = dense_R(2, 2, nz)
    P = R.T.copy()  # piecewise constant: every child takes its parent's value
    Ac = dense_from_apply(lambda x: orc.apply(g.coarse(), x), (nz, 1, 1))
    G = R @ A @ P
    assert np.abs(G - Ac).max() <= 1e-14 * np.abs(Ac).max()


@pytest.mark.parametrize("shape", [(8, 4, 5), (4, 8, 3), (6, 2, 4)])
def test_coarse_vertical_couplings_are_galerkin(orc, shape):
    """On any grid, the entries of R A P that join two different levels come
    from the vertical faces alone, so they must equal the coarse operator's:
    this fixes which four fine columns each coarse face sums."""
    nx, ny, nz = shape
    g, _ = grid3(orc, nx, ny, nz, seed=nx * ny, graded=True)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    R = dense_R(nx, ny, nz)
    G = R @ A @ R.T
    gc = g.coarse()
    Ac = dense_from_apply(lambda x: orc.apply(gc, x), gc.shape)
    ncol = (nx // 2) * (ny // 2)
    kk = np.arange(nz * ncol) // ncol
    across = kk[:, None] != kk[None, :]
    assert np.abs(Ac[across]).max() > 0
    assert np.abs(G[across] - Ac[across]).max() <= 1e-14 * np.abs(Ac).max()


def face_assembly(nx, ny, nz, hx, hy, omega2, dz, lam3):
    """Dense A assembled face by face: every face adds its coefficient to the
    two cells' diagonals and subtracts it from their coupling."""
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = lambda i, j, k: (k * ny + (j % ny)) * nx + (i % nx)  # noqa: E731
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                A[idx(i, j, k), idx(i, j, k)] += hx * hy * dz[k]
    faces = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if nx > 1:
                    faces.append((idx(i, j, k), idx(i + 1, j, k), omega2 * hy * dz[k] / hx))
                if ny > 1:
                    faces.append((idx(i, j, k), idx(i, j + 1, k), omega2 * hx * dz[k] / hy))
                if k + 1 < nz:
                    half = dz[k] / (2 * lam3[k, j, i]) + dz[k + 1] / (2 * lam3[k + 1, j, i])
                    faces.append((idx(i, j, k), idx(i, j, k + 1), omega2 * hx * hy / half))
    for a, b, t in faces:
        A[a, a] += t
        A[b, b] += t
        A[a, b] -= t
        A[b, a] -= t
    return A


@pytest.mark.parametrize("shape", [(4, 4, 3), (4, 2, 4), (2, 4, 3), (1, 4, 3), (4, 1, 3), (1, 1, 5)])
def test_dense_operator_symmetric_positive_and_face_assembled(orc, shape):
    nx, ny, nz = shape
    g, lam3 = grid3(orc, nx, ny, nz, seed=sum(shape))
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    B = face_assembly(nx, ny, nz, g.hx, g.hy, g.omega2, g.dz, lam3)
    assert np.abs(A - B).max() <= 1e-14 * np.abs(A).max()


def test_symmetry_and_positivity_on_a_graded_grid(orc):
    g, _ = grid3(orc, 16, 8, 24, seed=4, graded=True)
    rng = np.random.default_rng(9)
    for _ in range(3):
        u, v = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
        uAv, vAu = float((u * orc.apply(g, v)).sum()), float((v * orc.apply(g, u)).sum())
        scale = float((np.abs(u) * orc.apply_abs(g, np.abs(v))).sum())
        assert abs(uAv - vAu) <= 1e-13 * scale
        assert float((u * orc.apply(g, u)).sum()) > 0


@pytest.mark.parametrize("nz", [1, 7, 40])
def test_one_column_sweep_is_the_exact_solve(orc, nz):
    g, _ = grid3(orc, 1, 1, nz, seed=nz)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    b = np.random.default_rng(nz).standard_normal(g.shape)
    u = orc.smooth_colour(g, 0, b, np.zeros(g.shape))
    ref = np.linalg.solve(A, b.ravel())
    assert np.abs(u.ravel() - ref).max() <= 1e-10 * np.abs(ref).max()


def test_sweep_zeroes_the_residual_of_its_colour(orc):
    """After a colour-c sweep (rho = 1) the residual vanishes on every column
    of colour c: each column's own tridiagonal system is solved exactly."""
    g, _ = grid3(orc, 8, 6, 10, seed=1)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(g.shape)
    u = rng.standard_normal(g.shape)
    j, i = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    for c in (0, 1):
        u = orc.smooth_colour(g, c, b, u)
        r = orc.residual(g, b, u)
        own = np.broadcast_to(((i + j) % 2) == c, g.shape)
        scale = np.abs(orc.apply_abs(g, u)).max() + np.abs(b).max()
        assert np.abs(r[own]).max() <= 1e-12 * scale


@pytest.mark.parametrize("shape,levels", [((4, 4, 4), 2), ((8, 4, 3), 3), ((8, 8, 2), 0)])
def test_pcg_converges_to_the_dense_solution(orc, shape, levels):
    nx, ny, nz = shape
    g, _ = grid3(orc, nx, ny, nz, seed=7, n_levels=levels)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    f = np.random.default_rng(1).standard_normal(g.shape)
    V = (g.hx * g.hy * g.dz)[:, None, None] * np.ones(g.shape)
    ref = np.linalg.solve(A, (V * f).ravel()).reshape(g.shape)
    for flexible in (True, False):
        u, st = orc.pcg(g, f, rtol=1e-13, flexible=flexible)
        assert st["status"] == 0
        assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape,levels,nus", [((8, 8, 4), 2, (1, 1, 1)), ((8, 4, 3), 3, (2, 1, 3)),
                                               ((4, 4, 5), 3, (1, 2, 5))])
def test_vcycle_matches_the_dense_recursion(orc, shape, levels, nus):
    """The V-cycle against Alg. "Multigrid V-cycle" written with dense matrices,
    the coarse operators being those of the coarsened faces."""
    nx, ny, nz = shape
    g, _ = grid3(orc, nx, ny, nz, seed=nx + nz, n_levels=levels, nu_pre=nus[0], nu_post=nus[1],
                 nu_coarse=nus[2])
    grids = [g]
    for _ in range(levels - 1):
        grids.append(grids[-1].coarse())
    As = [dense_from_apply(lambda x, gg=gg: orc.apply(gg, x), gg.shape) for gg in grids]
    b = np.random.default_rng(6).standard_normal(g.shape)
    ref = dense_vcycle(grids, As, b, *nus)
    np.testing.assert_allclose(orc.vcycle(g, b), ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())


def test_vcycle_with_constant_prolongation_is_spd(orc):
    """Down to one column (an exact coarse solve), P = R^T and the reversed
    post-smoothing order make the V-cycle symmetric positive definite."""
    g, _ = grid3(orc, 4, 4, 3, seed=2, prolong=1)
    B = dense_from_apply(lambda r: orc.vcycle(g, r), g.shape)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    # and it contracts: the spectral radius of I - B A is below one
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    assert np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - B @ A)).max() < 1.0
