"""GPU parity on deep columns and the colour discipline of the rho = 1 sweeps.

Deep columns: the paper's runs use 128 vertical levels and mentions 256
(Sec. 7.1).  Columns of 129..256 levels take the four 64-level k-segment
kernels on the finest level, deeper ones the sequential column kernel (the
mixed-precision solve then runs the plain FP32 V-cycle on a cast copy of
the residual; the batch engine takes at most 256 levels).

Colour discipline (Sec. 4.2 eq. BlockRBSOR with rho = 1): a half-sweep of
colour c overwrites the colour-c columns without reading their old values,
a colour-0-only prolongation leaves colour 1 alone, and the restriction
right after a colour-1 sweep takes the colour-0 residual only.  NaN placed in
exactly the values that must not be read may not reach any output.
"""
import numpy as np
import pytest
import torch

from helpers import small_grid
from solve_parity import check_solve
from paper_1307_2036_amd import inputs as I

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def ell():
    from paper_1307_2036_amd import ell as E
    E.load_library()
    assert torch.cuda.is_available()
    return E


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_grid(ell, g, precision="fp64"):
    return ell.Grid(g.nx, g.ny, g.nz, g.hx, g.hy, g.omega2, g.dz, g.lambda2, g.n_levels, g.nu_pre,
                    g.nu_post, g.nu_coarse, g.rho, g.prolong, precision)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def zeros(shape):
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


DEEP = [(32, 16, 192), (16, 16, 256), (16, 8, 300)]


@pytest.mark.parametrize("shape", DEEP)
def test_deep_column_kernels(ell, orc, shape):
    """Operator, both colours of line relaxation (from zero and from a
    non-zero start) on every level, and one V-cycle, against the oracle."""
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=nz)
    G = gpu_grid(ell, g)
    rng = np.random.default_rng(nz)
    x = rng.standard_normal(g.shape)
    y = host(G.apply_A(dev(x)))
    assert np.all(np.abs(y - orc.apply(g, x)) <= 16 * EPS * orc.apply_abs(g, x))
    gl = g
    for lv in range(G.levels):
        b = rng.standard_normal(gl.shape) * (gl.hx * gl.hy * gl.dz)[:, None, None]
        bs = G.to_split(lv, dev(b))
        us = G.level_empty(lv)
        G.level_smooth(lv, 0, bs, us, zero_init=True)
        G.level_smooth(lv, 1, bs, us)
        G.level_smooth(lv, 0, bs, us)
        ref = orc.smooth_colour(gl, 0, b, orc.smooth_colour(gl, 1, b, orc.smooth_colour(
            gl, 0, b, np.zeros(gl.shape))))
        got = host(G.from_split(lv, us, zeros(gl.shape)))
        scale = np.abs(ref).max(axis=0, keepdims=True)
        assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300), (lv, np.abs(got - ref).max())
        if lv + 1 < G.levels:
            gl = gl.coarse()
    r = rng.standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    assert rel(host(G.vcycle(dev(r))), orc.vcycle(g, r)) <= 1e-11


@pytest.mark.parametrize("shape", DEEP)
def test_deep_column_solves(ell, orc, shape):
    """Whole solves, both betas, on the paper's level placement.  (With the
    quadratic grading over depth 1/50 the vertical couplings at 192 levels
    exceed the cell volumes by ~1e30: the FP64 true residual of the oracle's
    own solution is 3% of ||b||, and rounding alone moves the stopping count
    of the recurrence by two, while the iterates still agree to 4e-16.)"""
    nx, ny, nz = shape
    p = I.paper_graded_problem(f"deep{nz}", nx, ny, nz, 1e-2, 63 + nz, 62 + nz)
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p)
    for flexible in (True, False):
        u, st = G.pcg_solve(dev(p.f), rtol=p.rtol, flexible=flexible)
        assert st.status == 0
        info = check_solve(orc, g, p.f, host(u), st, p.rtol, flexible=flexible)
        print(shape, "flexible" if flexible else "classic", info)


@pytest.mark.parametrize("shape", DEEP)
@pytest.mark.parametrize("precision", ["fp32", "bf16coef"])
def test_deep_column_mixed_tight_solve(ell, orc, shape, precision):
    """Validation mode (rtol 1e-12) of the mixed-precision solve against the
    oracle's tight solve.  Up to 256 levels the finest level runs the hybrid
    V-cycle (FP32 pre-smoothing reading the FP64 residual through the segment
    kernels, FP64 post-smoothing); deeper columns fall back to the plain FP32
    V-cycle on a cast copy of the residual (column kernels), there on uniform
    levels, whose column systems FP32 resolves (on graded ones the plain FP32
    V-cycle is no useful preconditioner, which is why the hybrid one exists)."""
    nx, ny, nz = shape
    if nz <= 256:
        p = I.paper_graded_problem(f"deepm{nz}", nx, ny, nz, 1e-2, 73 + nz, 72 + nz)
    else:
        g0 = small_grid(orc, nx, ny, nz, graded=False, seed=nz, omega2=1e-2)
        p = I.Problem("deepm300", nx, ny, nz, g0.hx, g0.hy, g0.dz, g0.lambda2, g0.omega2,
                      I.rhs_normal(nx, ny, g0.dz, 73 + nz))
    g = orc.Grid.from_problem(p)
    u_ref, _ = orc.pcg(g, p.f, rtol=1e-12, maxiter=400)
    G = ell.Grid.from_problem(p, precision=precision)
    if nz > 256:  # the plain FP32 V-cycle: none of the hybrid path's fused forms
        assert not any(G.features.values()), G.features
    u, st = G.pcg_solve(dev(p.f), rtol=1e-12, maxiter=400)
    assert st.status == 0, st
    print(shape, precision, "iters", st.iters, "rel", rel(host(u), u_ref))
    assert rel(host(u), u_ref) <= 1e-8


def test_batch_rejects_columns_deeper_than_256(ell):
    p = I.graded_problem("deep300", 16, 300, 1e-2, 1, 2, with_f=False)
    B = ell.Batch(1 << 30)
    for precision in ("fp64", "fp32"):
        with pytest.raises(ell.EllError) as e:
            B.grid(p, precision=precision)
        assert e.value.code == ell.ELL_ERR_INVALID
    B.close()


def colour_mask(nx, ny):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return (i + j) % 2


# finest and coarse levels; tiled and column kernels (nx/2 odd takes the
# column kernel: 34 x 10 on its only level, 68 x 12 on its coarse 34 x 6
# level); 4, 8 and 16 k-segments; one-wide grids; deep columns
POISON_SHAPES = [((64, 32, 24), 3), ((34, 10, 100), 1), ((68, 12, 100), 2), ((128, 64, 128), 4),
                 ((6, 1, 5), 1), ((1, 6, 4), 1), ((16, 8, 300), 2)]


@pytest.mark.parametrize("tile", [1, 0])
@pytest.mark.parametrize("shape,levels", POISON_SHAPES)
def test_sweep_never_reads_its_own_colour(ell, orc, shape, levels, tile):
    """rho = 1: NaN in the old values of the colour being swept never reaches
    the output, which equals the sweep from zeroed own-colour values bitwise;
    every level and both colours."""
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=3 * nx + nz, n_levels=levels)
    ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, tile)
    try:
        G = gpu_grid(ell, g)
    finally:
        ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, 1)
    rng = np.random.default_rng(nx + nz)
    gl = g
    for lv in range(G.levels):
        mask = colour_mask(gl.nx, gl.ny)
        b = rng.standard_normal(gl.shape) * (gl.hx * gl.hy * gl.dz)[:, None, None]
        u = rng.standard_normal(gl.shape) * 1e-3
        bs = G.to_split(lv, dev(b))
        for c in (0, 1):
            own = np.broadcast_to(mask == c, gl.shape)
            clean = np.where(own, 0.0, u)
            poisoned = np.where(own, np.nan, u)
            out = []
            for start in (clean, poisoned):
                us = G.to_split(lv, dev(start))
                G.level_smooth(lv, c, bs, us)
                out.append(host(G.from_split(lv, us, zeros(gl.shape))))
            assert np.all(np.isfinite(out[1])), (lv, c)
            np.testing.assert_array_equal(out[1], out[0])
        if lv + 1 < G.levels:
            gl = gl.coarse()


@pytest.mark.parametrize("shape", [(64, 32, 24), (68, 12, 100), (4, 4, 70), (16, 8, 300)])
def test_red_only_prolongation_and_black_zero_restriction_skip_poison(ell, orc, shape):
    """The colour-0-only prolongation neither reads nor writes colour 1 (NaN
    there stays put and reaches no colour-0 value), and the restriction after
    a colour-1 sweep never reads colour 1 of the right-hand side."""
    nx, ny, nz = shape
    g = small_grid(orc, nx, ny, nz, seed=nx + 5 * nz, n_levels=2)
    G = gpu_grid(ell, g)
    rng = np.random.default_rng(nz)
    black = np.broadcast_to(colour_mask(nx, ny) == 1, g.shape)
    u = rng.standard_normal(g.shape)
    uc = rng.standard_normal((nz, ny // 2, nx // 2))
    ucs = G.to_split(1, dev(uc))
    out = []
    for start in (np.where(black, 0.0, u), np.where(black, np.nan, u)):
        us = G.to_split(0, dev(start))
        G.level_prolong_add(0, ucs, us, red_only=True)
        out.append(host(G.from_split(0, us, zeros(g.shape))))
    assert np.all(np.isnan(out[1][black]))
    np.testing.assert_array_equal(out[1][~black], out[0][~black])
    # restriction right after a red, black sweep pair, with NaN in the black b
    b = rng.standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    bs = G.to_split(0, dev(b))
    us = G.level_empty(0)
    G.level_smooth(0, 0, bs, us, zero_init=True)
    G.level_smooth(0, 1, bs, us)
    res = []
    for bb in (b, np.where(black, np.nan, b)):
        bc = G.level_empty(1)
        G.level_resid_restrict(0, G.to_split(0, dev(bb)), us, bc, black_zero=True)
        res.append(host(G.from_split(1, bc, zeros((nz, ny // 2, nx // 2)))))
    assert np.all(np.isfinite(res[1]))
    np.testing.assert_array_equal(res[1], res[0])
