"""Pins of the multigrid V-cycle (Sec. 4.3 Alg. "Multigrid V-cycle", tensor-
product variant of Sec. 4.3.1 / 6.2.1) used as the preconditioner."""
import numpy as np
import pytest

from helpers import dense_from_apply, small_grid
from test_oracle_smoother import block_sor_dense


def dense_R(nx, ny, nz):
    nxc, nyc = nx // 2, ny // 2
    R = np.zeros((nz * nyc * nxc, nz * ny * nx))
    for k in range(nz):
        for J in range(nyc):
            for I in range(nxc):
                for b in range(2):
                    for a in range(2):
                        R[(k * nyc + J) * nxc + I, (k * ny + 2 * J + b) * nx + 2 * I + a] = 1.0
    return R


def dense_P_bilinear(nx, ny, nz):
    nxc, nyc = nx // 2, ny // 2
    P = np.zeros((nz * ny * nx, nz * nyc * nxc))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                I, J = i // 2, j // 2
                I2 = (I + (1 if i % 2 else -1)) % nxc
                J2 = (J + (1 if j % 2 else -1)) % nyc
                row = (k * ny + j) * nx + i
                for (ii, jj, w) in [(I, J, 9), (I2, J, 3), (I, J2, 3), (I2, J2, 1)]:
                    P[row, (k * nyc + jj) * nxc + ii] += w / 16.0
    return P


def dense_vcycle(grids, As, b, nu_pre, nu_post, nu_coarse, level=0):
    g, A = grids[level], As[level]
    u = np.zeros(g.shape)
    if level == len(grids) - 1:
        for _ in range(nu_coarse):
            u = block_sor_dense(A, g.shape, 0, 1.0, b, u)
            u = block_sor_dense(A, g.shape, 1, 1.0, b, u)
        return u
    for _ in range(nu_pre):
        u = block_sor_dense(A, g.shape, 0, 1.0, b, u)
        u = block_sor_dense(A, g.shape, 1, 1.0, b, u)
    r = b.ravel() - A @ u.ravel()
    gc = grids[level + 1]
    bc = (dense_R(g.nx, g.ny, g.nz) @ r).reshape(gc.shape)
    uc = dense_vcycle(grids, As, bc, nu_pre, nu_post, nu_coarse, level + 1)
    u = u + (dense_P_bilinear(g.nx, g.ny, g.nz) @ uc.ravel()).reshape(g.shape)
    for _ in range(nu_post):
        u = block_sor_dense(A, g.shape, 1, 1.0, b, u)
        u = block_sor_dense(A, g.shape, 0, 1.0, b, u)
    return u


@pytest.mark.parametrize("shape,levels,nus", [
    ((8, 8, 4), 2, (1, 1, 1)),
    ((8, 8, 3), 4, (1, 1, 1)),
    ((8, 4, 3), 3, (2, 1, 3)),
    ((4, 4, 5), 3, (1, 2, 5)),
])
def test_vcycle_matches_dense_recursion(orc, shape, levels, nus):
    nx, ny, nz = shape
    nu_pre, nu_post, nu_coarse = nus
    g = small_grid(orc, nx, ny, nz, seed=nx * ny + nz, n_levels=levels, nu_pre=nu_pre,
                   nu_post=nu_post, nu_coarse=nu_coarse)
    assert orc.num_levels(g) == levels
    grids = [g]
    for _ in range(levels - 1):
        grids.append(grids[-1].coarse())
    As = [dense_from_apply(lambda x, gg=gg: orc.apply(gg, x), gg.shape) for gg in grids]
    b = np.random.default_rng(6).standard_normal(g.shape)
    ref = dense_vcycle(grids, As, b, nu_pre, nu_post, nu_coarse)
    got = orc.vcycle(g, b)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())


def test_vcycle_is_linear(orc):
    g = small_grid(orc, 16, 16, 8, seed=2)
    rng = np.random.default_rng(1)
    r1, r2 = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    z = orc.vcycle(g, 2.0 * r1 - 3.0 * r2)
    ref = 2.0 * orc.vcycle(g, r1) - 3.0 * orc.vcycle(g, r2)
    np.testing.assert_allclose(z, ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())


def test_symmetric_variant_is_spd_and_contracts(orc):
    """With piecewise-constant prolongation (P = R^T) and post-smoothing in the
    reverse colour order the V-cycle is a symmetric positive definite operator
    B, and the error propagator I - BA contracts."""
    g = small_grid(orc, 4, 4, 4, seed=5, prolong=1)
    B = dense_from_apply(lambda x: orc.vcycle(g, x), g.shape)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    np.testing.assert_allclose(B, B.T, rtol=1e-9, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    E = np.eye(A.shape[0]) - B @ A
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0


def test_bilinear_vcycle_contracts(orc):
    g = small_grid(orc, 8, 8, 4, seed=8)
    B = dense_from_apply(lambda x: orc.vcycle(g, x), g.shape)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    assert np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - B @ A)).max() < 0.5


def test_single_column_vcycle_is_exact(orc):
    g = small_grid(orc, 1, 1, 17, seed=1)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    r = np.random.default_rng(3).standard_normal(g.shape)
    np.testing.assert_allclose(orc.vcycle(g, r).ravel(), np.linalg.solve(A, r.ravel()), rtol=1e-10)


def test_too_many_levels_rejected(orc):
    g = small_grid(orc, 8, 8, 2, n_levels=5)
    with pytest.raises(ValueError):
        orc.vcycle(g, np.zeros(g.shape))
