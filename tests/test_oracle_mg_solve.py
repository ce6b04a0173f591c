"""Oracle pins for the stand-alone multigrid solver (Sec. 4.3: the V-cycle
iterated as a solver, u <- u + M(b - A u); Sec. 7.3, Table 3).

Independent pins: converged solves equal numpy's dense solve; a single column
converges in one iteration (the V-cycle on one column is the exact column
solve); the iteration count obeys the contraction of the dense error
propagator I - M A (its spectral radius from numpy's eigenvalues of the dense
matrices); in the paper's regime the iteration count is that of Table 3 (6)
within a tolerance and does not depend on lambda^2 (Table 6).
"""
import math

import numpy as np
import pytest

from helpers import dense_from_apply, small_grid
from paper_1307_2036_amd import inputs as I


@pytest.mark.parametrize("shape", [(4, 4, 3), (6, 4, 5), (8, 8, 4)])
def test_converged_solve_equals_dense_solve(orc, shape):
    g = small_grid(orc, *shape, seed=sum(shape), graded=False)
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    f = np.random.default_rng(4).standard_normal(g.shape)
    b = (g.hx * g.hy * g.dz)[:, None, None] * f
    ref = np.linalg.solve(A, b.ravel()).reshape(g.shape)
    u, st = orc.mg_solve(g, f, rtol=1e-13, maxiter=200)
    assert st["status"] == 0
    assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(st["true_r_norm"] - st["r_norm"]) <= 1e-11 * st["r0_norm"]


def test_single_column_in_one_iteration(orc):
    g = small_grid(orc, 1, 1, 30, seed=3, graded=False)
    f = np.random.default_rng(5).standard_normal(g.shape)
    u, st = orc.mg_solve(g, f, rtol=1e-12)
    assert st["iters"] == 1 and st["status"] == 0


def test_iterations_follow_the_dense_contraction_rate(orc):
    g = small_grid(orc, 8, 8, 4, seed=9, graded=False)
    n = g.nx * g.ny * g.nz
    A = dense_from_apply(lambda x: orc.apply(g, x), g.shape)
    M = dense_from_apply(lambda r: orc.vcycle(g, r), g.shape)
    rho = max(abs(np.linalg.eigvals(np.eye(n) - M @ A)))
    assert 0.0 < rho < 0.5
    f = np.random.default_rng(6).standard_normal(g.shape)
    u, st = orc.mg_solve(g, f, rtol=1e-8)
    bound = math.ceil(math.log(1e-8) / math.log(rho))
    assert 1 <= st["iters"] <= bound + 3, (st["iters"], bound, rho)


def paper_like(orc, nx, lam_factor=1.0):
    nz = 128
    h = math.pi / (2 * nx)
    dz = I.dz_paper_grading(nz, 0.01)
    lam = np.full(nz, I.paper_lambda2(600.0) * lam_factor)
    return orc.Grid(nx, nx, nz, h, h, 17.8 * h * h, dz, lam)


def test_soft_pin_paper_regime_iterations_and_lambda_independence(orc):
    its = []
    for lf in (1e-2, 1.0, 1e2):
        g = paper_like(orc, 64, lf)
        u, st = orc.mg_solve(g, I.rhs_normal(64, 64, g.dz, 5), rtol=1e-5)
        assert st["status"] == 0
        its.append(st["iters"])
    assert all(3 <= k <= 9 for k in its), its   # Table 3 prints 6
    assert max(its) - min(its) <= 1, its       # Table 6: independent of lambda^2
