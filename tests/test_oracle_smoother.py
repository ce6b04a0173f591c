"""Pins of the block (vertical line) red/black SOR smoother (Sec. 4.2 eq.
BlockRBSOR, Sec. 6.2.1) by brute force on dense matrices."""
import numpy as np
import pytest

from helpers import colour_columns, dense_from_apply, small_grid


def block_sor_dense(A, shape, colour, rho, b, u):
    """One colour of block SOR written with dense linear algebra: every column
    of the colour is solved from the dense rows of A with all other unknowns
    moved to the right-hand side."""
    nz, ny, nx = shape
    u = u.ravel().copy()
    b = b.ravel()
    new = u.copy()
    for (i, j) in colour_columns(nx, ny, colour):
        rows = np.array([(k * ny + j) * nx + i for k in range(nz)])
        others = np.setdiff1d(np.arange(u.size), rows)
        rhs = b[rows] - A[np.ix_(rows, others)] @ u[others]
        w = np.linalg.solve(A[np.ix_(rows, rows)], rhs)
        new[rows] = (1 - rho) * u[rows] + rho * w
    return new.reshape(shape)


@pytest.mark.parametrize("shape", [(4, 4, 5), (2, 2, 3), (4, 2, 3), (1, 4, 4), (6, 4, 2), (2, 1, 5)])
@pytest.mark.parametrize("rho", [1.0, 0.7])
def test_smoother_matches_dense_block_sor(orc, shape, rho):
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=nx + 10 * ny)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(g.shape)
    u = rng.standard_normal(g.shape)
    for colour in (0, 1):
        got = orc.smooth_colour(g, colour, b, u, rho)
        ref = block_sor_dense(A, g.shape, colour, rho, b, u)
        scale = np.abs(ref).max()
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-11 * scale)
        # columns of the other colour are untouched
        other = np.array([[(i + j) % 2 != colour for i in range(nx)] for j in range(ny)])
        np.testing.assert_array_equal(got[:, other], u[:, other])


def test_black_residual_zero_after_sweep(orc):
    """After red then black with rho = 1, every black column satisfies its
    equations exactly (up to rounding)."""
    g = small_grid(orc, 8, 8, 16, seed=4)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    u = orc.smooth_colour(g, 0, b, np.zeros(g.shape))
    u = orc.smooth_colour(g, 1, b, u)
    r = orc.residual(g, b, u)
    scale = orc.apply_abs(g, u) + np.abs(b)
    black = np.array([[(i + j) % 2 == 1 for i in range(8)] for j in range(8)])
    assert np.all(np.abs(r[:, black]) <= 1e-13 * scale[:, black])
    assert np.abs(r[:, ~black]).max() > 1e3 * np.abs(r[:, black]).max()


def test_exact_solution_is_fixed_point(orc):
    g = small_grid(orc, 4, 4, 6, seed=9)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(g.shape)
    u = np.linalg.solve(A, b.ravel()).reshape(g.shape)
    for colour in (0, 1):
        np.testing.assert_allclose(orc.smooth_colour(g, colour, b, u), u, rtol=1e-9,
                                   atol=1e-10 * np.abs(u).max())


def test_single_column_one_sweep_exact(orc):
    """One column: a sweep is the exact solve (moderate coefficients, so that the
    dense LU reference is itself accurate; the extreme range is pinned against
    rational arithmetic in the column-solve tests)."""
    g = small_grid(orc, 1, 1, 20, seed=3, graded=False)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    b = np.random.default_rng(0).standard_normal(g.shape)
    u = orc.smooth_colour(g, 0, b, np.zeros(g.shape))
    np.testing.assert_allclose(u.ravel(), np.linalg.solve(A, b.ravel()), rtol=1e-10)
