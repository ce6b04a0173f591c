"""Pins of restriction and prolongation (Sec. 4.3 "Intergrid operators",
Sec. 6.2.1: cell average and linear interpolation)."""
import numpy as np
import pytest

from helpers import small_grid


@pytest.mark.parametrize("shape", [(8, 8, 3), (4, 2, 2), (2, 2, 4), (16, 4, 1)])
def test_restriction_sums_children(orc, shape):
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz)
    r = np.random.default_rng(0).standard_normal(g.shape)
    bc = orc.restrict(g, r)
    ref = r.reshape(nz, ny // 2, 2, nx // 2, 2).sum(axis=(2, 4))
    np.testing.assert_allclose(bc, ref, rtol=1e-15, atol=1e-15)
    np.testing.assert_array_equal(orc.restrict(g, np.ones(g.shape)), 4.0)


@pytest.mark.parametrize("mode", [0, 1])
def test_prolongation_preserves_constants(orc, mode):
    g = small_grid(orc, 8, 4, 3)
    u = orc.prolong_add(g, np.full((3, 2, 4), 2.5), np.zeros(g.shape), mode)
    np.testing.assert_allclose(u, 2.5, rtol=1e-15)


def test_bilinear_reproduces_bilinear_functions(orc):
    """Cell-centred bilinear interpolation is exact for a + bx + cy + dxy
    wherever the stencil does not wrap around the periodic boundary."""
    g = small_grid(orc, 16, 12, 2)
    nxc, nyc = 8, 6
    Xc = (np.arange(nxc) + 0.5) * 2
    Yc = (np.arange(nyc) + 0.5) * 2
    fn = lambda x, y: 0.3 + 1.7 * x - 0.4 * y + 0.25 * x * y
    uc = np.broadcast_to(fn(Xc[None, :], Yc[:, None]), (2, nyc, nxc)).copy()
    u = orc.prolong_add(g, uc, np.zeros(g.shape), 0)
    Xf = np.arange(16) + 0.5
    Yf = np.arange(12) + 0.5
    ref = fn(Xf[None, :], Yf[:, None])
    inner = (slice(1, 11), slice(1, 15))
    np.testing.assert_allclose(u[0][inner], ref[inner], rtol=1e-13)
    np.testing.assert_allclose(u[1][inner], ref[inner], rtol=1e-13)


def test_prolongation_adds(orc):
    g = small_grid(orc, 4, 4, 2)
    rng = np.random.default_rng(1)
    uc = rng.standard_normal((2, 2, 2))
    u0 = rng.standard_normal(g.shape)
    a = orc.prolong_add(g, uc, u0, 0)
    b = orc.prolong_add(g, uc, np.zeros(g.shape), 0)
    np.testing.assert_allclose(a, u0 + b, rtol=1e-14, atol=1e-14)


def test_bilinear_weights_periodic(orc):
    """A coarse unit spike spreads with weights 9,3,3,1 (/16) to the fine cells
    around it, including across the periodic wrap."""
    g = small_grid(orc, 4, 4, 1)
    uc = np.zeros((1, 2, 2))
    uc[0, 0, 0] = 16.0
    u = orc.prolong_add(g, uc, np.zeros(g.shape), 0)[0]
    # on a 2-cell coarse grid I-1 and I+1 are the same cell, so the 3/16 and
    # 1/16 weights of both sides land on the other coarse cell
    expect = np.zeros((4, 4))
    for j in range(4):
        for i in range(4):
            wx = 0.75 if i // 2 == 0 else 0.25
            wy = 0.75 if j // 2 == 0 else 0.25
            expect[j, i] = 16 * wx * wy
    np.testing.assert_allclose(u, expect, rtol=1e-15)


def test_constant_prolongation_is_restriction_transpose(orc):
    g = small_grid(orc, 8, 4, 3)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(g.shape)
    ec = rng.standard_normal((3, 2, 4))
    lhs = float((orc.restrict(g, r) * ec).sum())
    rhs = float((r * orc.prolong_add(g, ec, np.zeros(g.shape), 1)).sum())
    assert abs(lhs - rhs) < 1e-13 * np.abs(r).sum()
