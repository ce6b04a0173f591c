"""Pins of the outer preconditioned CG loop (Appendix B, Alg. "Preconditioned
Conjugate Gradient method", with the residual update r <- r - alpha q)."""
import numpy as np
import pytest

from helpers import closed_form_mu, dense_from_apply, mode, small_grid, volumes
from paper_1307_2036_amd import inputs as I


@pytest.mark.parametrize("shape,flexible", [((8, 8, 6), True), ((8, 8, 6), False),
                                             ((4, 2, 9), True), ((16, 16, 4), True)])
def test_tight_solve_equals_dense_solve(orc, shape, flexible):
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=nz)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    f = np.random.default_rng(0).standard_normal(g.shape)
    b = volumes(g) * f
    ref = np.linalg.solve(A, b.ravel()).reshape(g.shape)
    u, st = orc.pcg(g, f, rtol=1e-13, maxiter=200, flexible=flexible)
    assert st["status"] == 0
    assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)


def test_eigenmode_rhs(orc):
    """With f = phi (an eigenvector, A phi = V mu phi) the solution is phi / mu."""
    g = small_grid(orc, 16, 8, 8, graded=False, omega2=0.05)
    phi = mode(g, 3, 1, 2)
    u, st = orc.pcg(g, phi, rtol=1e-12, maxiter=100)
    np.testing.assert_allclose(u, phi / closed_form_mu(g, 3, 1, 2), rtol=0, atol=1e-11)


def test_single_column_converges_in_one_iteration(orc):
    """On one column the V-cycle is the exact column solve, so M^{-1} = A^{-1}
    (moderate coefficients keep the rounding of that solve below the tolerance)."""
    g = small_grid(orc, 1, 1, 30, seed=4, graded=False)
    f = np.random.default_rng(1).standard_normal(g.shape)
    u, st = orc.pcg(g, f, rtol=1e-12)
    assert st["iters"] == 1 and st["status"] == 0


def test_zero_rhs(orc):
    g = small_grid(orc, 8, 8, 4)
    u, st = orc.pcg(g, np.zeros(g.shape))
    assert st["iters"] == 0 and st["status"] == 0
    assert not u.any()


def test_volume_mean_is_conserved(orc):
    """1'A = V' (A 1 = V and A symmetric), so the exact solution satisfies
    sum V u = sum V f; the approximate one does up to the final residual."""
    g = small_grid(orc, 16, 16, 8, seed=3)
    f = np.random.default_rng(2).standard_normal(g.shape) + 0.3
    u, st = orc.pcg(g, f, rtol=1e-10, maxiter=100)
    V = volumes(g)
    assert abs((V * u).sum() - (V * f).sum()) <= 2 * st["r_norm"] * np.sqrt(u.size) + 1e-14 * np.abs(V * f).sum()


def test_maxiter_and_nan(orc):
    g = small_grid(orc, 16, 16, 8)
    f = np.random.default_rng(2).standard_normal(g.shape)
    u, st = orc.pcg(g, f, rtol=1e-12, maxiter=1)
    assert st["status"] == 1 and st["iters"] == 1
    f[0, 0, 0] = np.nan
    u, st = orc.pcg(g, f, rtol=1e-12, maxiter=5)
    assert st["status"] == -4


def test_warm_start_relative_to_rhs(orc):
    g = small_grid(orc, 16, 16, 8, seed=6)
    f = np.random.default_rng(3).standard_normal(g.shape)
    u, st = orc.pcg(g, f, rtol=1e-8, maxiter=100, rel_to_rhs=True)
    u2, st2 = orc.pcg(g, f, u0=u, rtol=1e-8, maxiter=100, rel_to_rhs=True)
    assert st2["iters"] == 0
    np.testing.assert_array_equal(u2, u)


def test_flexible_and_classic_beta_agree_for_symmetric_preconditioner(orc):
    """With P = R^T the V-cycle is symmetric, <z_K, r_{K-1}> = 0 in exact
    arithmetic and both beta formulas coincide."""
    g = small_grid(orc, 16, 16, 8, seed=2, prolong=1)
    f = np.random.default_rng(4).standard_normal(g.shape)
    u1, s1 = orc.pcg(g, f, rtol=1e-9, flexible=True)
    u2, s2 = orc.pcg(g, f, rtol=1e-9, flexible=False)
    assert s1["iters"] == s2["iters"]
    assert np.linalg.norm(u1 - u2) < 1e-8 * np.linalg.norm(u1)


def paper_like_grid(orc, O_nx=64, lam_factor=1.0, omega_factor=1.0):
    """Parameters of the paper's 256^2 x 128 run (Table 1) on a flat panel of
    n_x columns: C_horiz = omega^2/h^2 = 17.8 (Sec. 3.1.2), lambda^2 = 0.0332,
    the paper's vertical grading with H = 1/100, h = pi/(2 n_x)."""
    import math
    nx, nz = O_nx, 128
    h = math.pi / (2 * nx)
    dz = I.dz_paper_grading(nz, 0.01)
    omega2 = 17.8 * h * h * omega_factor
    lam = np.full(nz, I.paper_lambda2(600.0) * lam_factor)
    return orc.Grid(nx, nx, nz, h, h, omega2, dz, lam)


def test_soft_pin_iterations_paper_regime(orc):
    """Soft pin: the paper's stand-alone GMG needs 6 iterations for a 1e-5
    reduction at C_horiz ~ 17.8 (Table 3); used as a CG preconditioner on the
    flat analogue it should need no more (allow +-2)."""
    g = paper_like_grid(orc)
    f = I.rhs_normal(g.nx, g.ny, g.dz, 5)
    u, st = orc.pcg(g, f, rtol=1e-5)
    assert 2 <= st["iters"] <= 8, st


def test_soft_pin_lambda_independence(orc):
    """Iteration counts do not depend on lambda^2 (Sec. 7.3.2, Table 6)."""
    its = []
    for lf in (1e-2, 1.0, 1e2):
        g = paper_like_grid(orc, lam_factor=lf)
        f = I.rhs_normal(g.nx, g.ny, g.dz, 5)
        its.append(orc.pcg(g, f, rtol=1e-5)[1]["iters"])
    assert max(its) - min(its) <= 1, its
