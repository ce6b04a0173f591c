"""GPU parity: every kernel of the hot path and the whole solve, called
through the C ABI, against the FP64 oracle on the same seeded inputs.

Tolerances (FP64): the kernels evaluate the same formulas as the oracle in a
different association order and with fused multiply-adds, so a result may
differ from the oracle's by a few units of rounding of the terms that form
it.  Operator and residual values are compared against
c * eps * (sum of |terms|), column solves against c * eps times the column's
magnitude, whole solves in relative L2 (<= 1e-10, the same iteration count).
"""
import math

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


SHAPES = [(32, 32, 16), (64, 48, 37), (2, 2, 3), (1, 6, 4), (6, 1, 5), (1, 1, 5), (4, 2, 3),
          (130, 8, 7)]


def grid_for(orc, shape, seed=3, **mg):
    nx, ny, nz = shape
    return small_grid(orc, nx, ny, nz, seed=seed + nx + 7 * ny + 31 * nz, **mg)


def level_grids(g, levels):
    out = [g]
    for _ in range(levels - 1):
        out.append(out[-1].coarse())
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_split_layout_roundtrip(ell, orc, shape):
    g = grid_for(orc, shape)
    G = gpu_grid(ell, g)
    x = np.random.default_rng(0).standard_normal(g.shape)
    xs = G.to_split(0, dev(x))
    assert xs.numel() == G.level_elems(0)
    y = G.from_split(0, xs, torch.zeros(g.shape, dtype=torch.float64, device="cuda"))
    np.testing.assert_array_equal(host(y), x)
    # the layout is the documented one: colour c, level k, column m
    H, S, C = G.level_layout(0)
    assert H == (g.nx * g.ny + 1) // 2 and S >= H and C >= g.nz * S
    flat = host(xs)
    assert flat.size == 2 * C
    seen = np.zeros(flat.size, dtype=bool)
    for j in range(g.ny):
        for i in range(g.nx):
            c = (i + j) % 2
            m = j * (g.nx // 2) + i // 2 if g.nx > 1 else j // 2
            idx = c * C + np.arange(g.nz) * S + m
            np.testing.assert_array_equal(flat[idx], x[:, j, i])
            seen[idx] = True
    assert not flat[~seen].any()  # padding stays zero


@pytest.mark.parametrize("shape", SHAPES)
def test_apply_matches_oracle(ell, orc, shape):
    g = grid_for(orc, shape)
    G = gpu_grid(ell, g)
    x = np.random.default_rng(1).standard_normal(g.shape)
    y = host(G.apply_A(dev(x)))
    ref = orc.apply(g, x)
    bound = 16 * EPS * orc.apply_abs(g, x)
    assert np.all(np.abs(y - ref) <= bound)


# (34, 10, 100) and (66, 18, 64): eight k-segments on the finest level (ragged: 13 x 7 + 9);
# (68, 10, 100), (4, 6, 70), (64, 48, 37): the LDS-tiled half-sweep (nx/2 and ny even), with a
# partial tile (34 = 32 + 2 m-columns), eight and four ragged segments
@pytest.mark.parametrize("shape", [(32, 32, 16), (64, 48, 37), (2, 2, 3), (1, 6, 4), (6, 1, 5),
                                   (1, 1, 5), (130, 8, 7), (34, 10, 100), (66, 18, 64),
                                   (68, 10, 100), (4, 6, 70)])
@pytest.mark.parametrize("rho", [1.0, 0.8])
def test_smoother_matches_oracle(ell, orc, shape, rho):
    g = grid_for(orc, shape, rho=rho)
    G = gpu_grid(ell, g)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    u0 = rng.standard_normal(g.shape) * 1e-3
    bs = G.to_split(0, dev(b))
    # red from zero, then black, then red again (all three code paths)
    us = G.level_empty(0)
    G.level_smooth(0, 0, bs, us, zero_init=True)
    ref = orc.smooth_colour(g, 0, b, np.zeros(g.shape), rho)
    for colour, zero in ((1, False), (0, False)):
        G.level_smooth(0, colour, bs, us, zero_init=zero)
        ref = orc.smooth_colour(g, colour, b, ref, rho)
    got = host(G.from_split(0, us, torch.zeros(g.shape, dtype=torch.float64, device="cuda")))
    scale = np.abs(ref).max(axis=0, keepdims=True)
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300), np.abs(got - ref).max() / scale.max()
    # from a non-zero start as well
    us = G.to_split(0, dev(u0))
    G.level_smooth(0, 1, bs, us)
    ref = orc.smooth_colour(g, 1, b, u0, rho)
    got = host(G.from_split(0, us, torch.zeros(g.shape, dtype=torch.float64, device="cuda")))
    assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref).max(axis=0, keepdims=True) + 1e-300)


@pytest.mark.parametrize("shape", [(68, 10, 100), (64, 48, 37), (4, 6, 70), (128, 16, 128), (96, 4, 32)])
def test_tiled_half_sweep_equals_column_kernel(ell, orc, shape):
    """The LDS-tiled finest-level half-sweep computes every column from the same
    terms in the same order as the column kernel: bitwise equal results."""
    g = grid_for(orc, shape)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    out = []
    for tile in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, tile)
        try:
            G = gpu_grid(ell, g)
        finally:
            ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, 1)
        bs = G.to_split(0, dev(b))
        us = G.level_empty(0)
        G.level_smooth(0, 0, bs, us, zero_init=True)
        for colour in (1, 0, 1, 0):
            G.level_smooth(0, colour, bs, us)
        out.append(host(us))
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.parametrize("shape,levels", [((128, 64, 100), 4), ((136, 24, 37), 3), ((64, 64, 128), 4),
                                          ((256, 32, 64), 3)])
def test_tiled_half_sweep_on_coarse_levels_equals_column_kernel(ell, orc, shape, levels):
    """Coarser levels use the tiled half-sweep too (plain accesses, 4, 8 or 16
    k-segments by level size; a level with nx/2 odd falls back to the column
    kernel): bitwise equal to the column kernel on every level."""
    g = grid_for(orc, shape, n_levels=levels)
    gl = level_grids(g, levels)
    out = []
    for tile in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, tile)
        try:
            G = gpu_grid(ell, g)
        finally:
            ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, 1)
        res = []
        for l in range(1, levels):
            b = np.random.default_rng(9 + l).standard_normal(gl[l].shape)
            bs = G.to_split(l, dev(b))
            us = G.level_empty(l)
            G.level_smooth(l, 0, bs, us, zero_init=True)
            for colour in (1, 0, 1, 0):
                G.level_smooth(l, colour, bs, us)
            res.append(host(us))
        out.append(res)
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("shape", [(32, 32, 16), (64, 48, 37), (4, 2, 3), (2, 2, 6), (256, 12, 9)])
def test_residual_restriction_matches_oracle(ell, orc, shape):
    g = grid_for(orc, shape, n_levels=2)
    G = gpu_grid(ell, g)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(g.shape)
    u = rng.standard_normal(g.shape)
    bc = G.level_empty(1)
    G.level_resid_restrict(0, G.to_split(0, dev(b)), G.to_split(0, dev(u)), bc)
    got = host(G.from_split(1, bc, torch.zeros((g.nz, g.ny // 2, g.nx // 2), dtype=torch.float64,
                                               device="cuda")))
    ref = orc.restrict(g, orc.residual(g, b, u))
    scale = orc.restrict(g, orc.apply_abs(g, u) + np.abs(b))
    assert np.all(np.abs(got - ref) <= 16 * EPS * scale)


# (32, 32, 128), (64, 64, 100): small levels with deep columns run the
# restriction with 16 and 8 (ragged) k-segments per coarse column
@pytest.mark.parametrize("shape", [(64, 32, 24), (32, 32, 128), (64, 64, 100)])
def test_black_zero_restriction_after_sweep(ell, orc, shape):
    """After red then black (rho = 1) the black residual is zero up to rounding,
    and the restriction that skips the black children agrees with the full one."""
    g = grid_for(orc, shape, n_levels=2)
    G = gpu_grid(ell, g)
    b = np.random.default_rng(5).standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    bs = G.to_split(0, dev(b))
    us = G.level_empty(0)
    G.level_smooth(0, 0, bs, us, zero_init=True)
    G.level_smooth(0, 1, bs, us)
    u = host(G.from_split(0, us, torch.zeros(g.shape, dtype=torch.float64, device="cuda")))
    bc = G.level_empty(1)
    G.level_resid_restrict(0, bs, us, bc, black_zero=True)
    got = host(G.from_split(1, bc, torch.zeros((g.nz, g.ny // 2, g.nx // 2), dtype=torch.float64,
                                               device="cuda")))
    ref = orc.restrict(g, orc.residual(g, b, u))
    scale = orc.restrict(g, orc.apply_abs(g, u) + np.abs(b))
    assert np.all(np.abs(got - ref) <= 64 * EPS * scale)


@pytest.mark.parametrize("shape", [(32, 32, 16), (64, 48, 37), (4, 2, 3), (2, 2, 6), (4, 4, 1),
                                   (32, 32, 128), (64, 64, 100)])
@pytest.mark.parametrize("mode", [0, 1])
def test_prolongation_matches_oracle(ell, orc, shape, mode):
    g = grid_for(orc, shape, n_levels=2, prolong=mode)
    G = gpu_grid(ell, g)
    rng = np.random.default_rng(6)
    uc = rng.standard_normal((g.nz, g.ny // 2, g.nx // 2))
    u = rng.standard_normal(g.shape)
    us = G.to_split(0, dev(u))
    G.level_prolong_add(0, G.to_split(1, dev(uc)), us)
    got = host(G.from_split(0, us, torch.zeros(g.shape, dtype=torch.float64, device="cuda")))
    ref = orc.prolong_add(g, uc, u, mode)
    np.testing.assert_allclose(got, ref, rtol=0, atol=8 * EPS * (np.abs(u).max() + np.abs(uc).max()))
    # red-only leaves black columns as they were
    us = G.to_split(0, dev(u))
    G.level_prolong_add(0, G.to_split(1, dev(uc)), us, red_only=True)
    got = host(G.from_split(0, us, torch.zeros(g.shape, dtype=torch.float64, device="cuda")))
    red = np.array([[(i + j) % 2 == 0 for i in range(g.nx)] for j in range(g.ny)])
    np.testing.assert_array_equal(got[:, ~red], u[:, ~red])
    np.testing.assert_allclose(got[:, red], ref[:, red], rtol=0,
                               atol=8 * EPS * (np.abs(u).max() + np.abs(uc).max()))


@pytest.mark.parametrize("shape", [(68, 12, 100), (4, 4, 70), (2, 2, 6), (132, 36, 7), (64, 64, 100)])
def test_tiled_prolongation_equals_column_kernel(ell, orc, shape):
    """The LDS-staged colour-0 bilinear prolongation combines the same four
    coarse values with the same weights in the same order: bitwise equal."""
    g = grid_for(orc, shape, n_levels=2)
    rng = np.random.default_rng(12)
    uc = rng.standard_normal((g.nz, g.ny // 2, g.nx // 2))
    u = rng.standard_normal(g.shape)
    out = []
    for tile in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, tile)
        try:
            G = gpu_grid(ell, g)
        finally:
            ell.set_tuning(ell.ELL_TUNE_SMOOTH_TILE, 1)
        us = G.to_split(0, dev(u))
        G.level_prolong_add(0, G.to_split(1, dev(uc)), us, red_only=True)
        out.append(host(us))
    np.testing.assert_array_equal(out[0], out[1])


def test_coarse_level_apply(ell, orc):
    g = grid_for(orc, (32, 16, 9), n_levels=3)
    G = gpu_grid(ell, g)
    for lv, gl in enumerate(level_grids(g, 3)):
        x = np.random.default_rng(lv).standard_normal(gl.shape)
        y = G.level_empty(lv)
        G.level_apply(lv, G.to_split(lv, dev(x)), y)
        got = host(G.from_split(lv, y, torch.zeros(gl.shape, dtype=torch.float64, device="cuda")))
        assert np.all(np.abs(got - orc.apply(gl, x)) <= 16 * EPS * orc.apply_abs(gl, x))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape,mg", [
    ((32, 32, 16), dict()),
    ((64, 64, 32), dict(n_levels=4, nu_coarse=5)),
    ((96, 96, 24), dict()),
    ((32, 16, 12), dict(nu_pre=2, nu_post=1, nu_coarse=3)),
    ((32, 32, 8), dict(rho=0.9)),
    ((32, 32, 8), dict(prolong=1)),
    ((32, 32, 8), dict(nu_pre=0, nu_post=2)),
    ((16, 16, 8), dict(nu_post=0)),
    ((1, 1, 12), dict()),
    ((32, 32, 8), dict(n_levels=1, nu_coarse=0)),         # block red/black SSOR (one level)
    ((16, 12, 7), dict(n_levels=2, nu_coarse=0)),
    ((20, 8, 6), dict(n_levels=1, nu_coarse=0, nu_pre=0, nu_post=2)),
])
def test_vcycle_matches_oracle(ell, orc, shape, mg):
    g = grid_for(orc, shape, **mg)
    G = gpu_grid(ell, g)
    assert G.levels == orc.num_levels(g)
    r = np.random.default_rng(7).standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    z = host(G.vcycle(dev(r)))
    ref = orc.vcycle(g, r)
    assert rel(z, ref) <= 1e-11


def test_config0_solve_matches_oracle(ell, orc):
    p = I.config0()
    g = orc.Grid.from_problem(p)
    u_ref, st_ref = orc.pcg(g, p.f, rtol=p.rtol)
    G = ell.Grid.from_problem(p)
    u, st = G.pcg_solve(dev(p.f), rtol=p.rtol)
    # uniform, moderately anisotropic grid: the stopping count is not rounding-sensitive
    assert st.status == 0 and st.iters == st_ref["iters"]
    assert rel(host(u), u_ref) <= 1e-10
    assert abs(st.r0_norm / st_ref["r0_norm"] - 1) < 1e-12
    assert abs(st.r_norm / st_ref["r_norm"] - 1) < 1e-6


@pytest.mark.parametrize("name,kw,opts", [
    ("graded64_L4", dict(nx=64, nz=32, n_levels=4, nu_coarse=5), dict()),
    ("graded96_std", dict(nx=96, nz=24), dict()),
    ("graded64_classic_beta", dict(nx=64, nz=16), dict(flexible=False)),
    ("graded128_tight", dict(nx=128, nz=64, n_levels=5, nu_coarse=5), dict(rtol=1e-10)),
])
def test_graded_solves_match_oracle(ell, orc, name, kw, opts):
    nx = kw.pop("nx")
    nz = kw.pop("nz")
    p = I.graded_problem(name, nx, nz, 1e-2, 11, 12, **kw)
    g = orc.Grid.from_problem(p)
    rtol = opts.pop("rtol", 1e-5)
    G = ell.Grid.from_problem(p)
    u, st = G.pcg_solve(dev(p.f), rtol=rtol, **opts)
    assert st.status == 0
    check_solve(orc, g, p.f, host(u), st, rtol, **opts)


# (64, 16, 32): whole tiles; (68, 12, 40): a partial tile (34 = 32 + 2 m-columns) and eight
# k-segments on the finest level; (128, 32, 64) with the mixed-precision V-cycle
@pytest.mark.parametrize("nx,ny,nz,levels,precision,flexible", [
    (64, 16, 32, 3, "fp64", False), (64, 16, 32, 3, "fp64", True), (68, 12, 100, 2, "fp64", True),
    (68, 12, 100, 2, "fp64", False), (128, 32, 64, 3, "fp32", True), (128, 32, 64, 3, "fp32", False)])
def test_fused_dots_equal_separate_pass(ell, orc, nx, ny, nz, levels, precision, flexible):
    """<r, z> (and <z, q>) formed by the last two post-smoothing half-sweeps give
    the iterates of the separate dot pass, up to the summation order: the same
    iteration count, solutions within 1e-10, both matching the oracle."""
    h = 1.0 / nx
    dz = I.dz_quadratic(nz, 1.0 / 50.0)
    p = I.Problem("fused", nx, ny, nz, h, h, dz, I.lambda2_perturbed(h, dz, 0.3, 22), 1e-2,
                  I.rhs_normal(nx, ny, dz, 21), n_levels=levels)
    res = []
    for fused in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_FUSED_DOT, fused)
        try:
            G = ell.Grid.from_problem(p, precision=precision)
        finally:
            ell.set_tuning(ell.ELL_TUNE_FUSED_DOT, 1)
        u, st = G.pcg_solve(dev(p.f), rtol=1e-8, flexible=flexible)
        assert st.status == 0
        res.append((host(u), st))
    (u1, s1), (u0, s0) = res
    assert s1.iters == s0.iters
    assert rel(u1, u0) <= 1e-10
    g = orc.Grid.from_problem(p)
    if precision == "fp64":
        check_solve(orc, g, p.f, u1, s1, 1e-8, flexible=flexible)
    else:
        u_ref, st_ref = orc.pcg(g, p.f, rtol=1e-8, flexible=flexible)
        assert s1.iters <= st_ref["iters"] + 2
        assert rel(u1, u_ref) <= 1e-6


@pytest.mark.parametrize("nx,ny,nz,levels,precision,flexible", [
    (64, 16, 32, 3, "fp64", False), (68, 12, 100, 2, "fp64", True), (64, 64, 48, 3, "fp64", False),
    (128, 32, 64, 3, "fp32", True), (68, 12, 40, 2, "fp32", False)])
def test_fused_update_equals_separate_pass(ell, orc, nx, ny, nz, levels, precision, flexible):
    """r -= alpha q and ||r||^2 carried by the first pre-smoothing pair (the
    convergence test between that pair and the rest of the V-cycle) give the
    iterates of the separate residual pass: the same iteration count, solutions
    within 1e-10, and the same final state at an iteration limit."""
    h = 1.0 / nx
    dz = I.dz_quadratic(nz, 1.0 / 50.0)
    p = I.Problem("fused_update", nx, ny, nz, h, h, dz, I.lambda2_perturbed(h, dz, 0.3, 24), 1e-2,
                  I.rhs_normal(nx, ny, dz, 23), n_levels=levels)
    res = []
    for fused in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_FUSED_UPDATE, fused)
        try:
            G = ell.Grid.from_problem(p, precision=precision)
        finally:
            ell.set_tuning(ell.ELL_TUNE_FUSED_UPDATE, 1)
        assert G.features["fused_update"] == bool(fused)
        u, st = G.pcg_solve(dev(p.f), rtol=1e-8, flexible=flexible)
        assert st.status == 0
        ul, stl = G.pcg_solve(dev(p.f), rtol=1e-14, maxiter=3, flexible=flexible)
        assert stl.status == ell.ELL_NOT_CONVERGED and stl.iters == 3
        res.append((host(u), st, host(ul), stl))
    (u1, s1, l1, t1), (u0, s0, l0, t0) = res
    assert s1.iters == s0.iters
    assert rel(u1, u0) <= 1e-10 and rel(l1, l0) <= 1e-10
    assert abs(t1.r_norm / t0.r_norm - 1) <= 1e-10
    if precision == "fp64":
        g = orc.Grid.from_problem(p)
        check_solve(orc, g, p.f, u1, s1, 1e-8, flexible=flexible)


@pytest.mark.parametrize("shape,mg", [((64, 64, 48), dict(n_levels=4, nu_coarse=5)),
                                      ((136, 16, 40), dict(n_levels=3)),
                                      ((128, 32, 100), dict(n_levels=4, nu_coarse=2, nu_post=2)),
                                      ((64, 8, 24), dict(n_levels=3))])
def test_coarse_prolongation_in_sweep_is_bitwise(ell, orc, shape, mg):
    """On the coarse levels the bilinear correction applied inside the first
    post-smoothing sweep adds the same four terms in the same order as the
    tiled prolongation pass: V-cycles with and without it are bitwise equal,
    and both match the oracle.  (136, 16): partial tiles on level 1 (hx2 =
    34); nu_post = 2: the later post-smoothing pairs follow the fused sweep;
    (64, 8): a two-row level 2 (coarse rows wrap onto themselves)."""
    g = grid_for(orc, shape, **mg)
    r = np.random.default_rng(11).standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    out = []
    for fused in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_FUSED_PROLONG, fused)
        try:
            G = gpu_grid(ell, g)
        finally:
            ell.set_tuning(ell.ELL_TUNE_FUSED_PROLONG, 1)
        assert G.features["coarse_prolong"] == bool(fused), G.features
        out.append(host(G.vcycle(dev(r))))
        G.close()
    assert np.array_equal(out[0], out[1])
    assert rel(out[0], orc.vcycle(g, r)) <= 1e-11


@pytest.mark.parametrize("shape,mg,precision", [
    ((128, 128, 128), dict(n_levels=5, nu_coarse=5), "fp64"),  # coarsest 8 x 8: the ring wraps onto the tile
    ((256, 128, 128), dict(n_levels=4, nu_coarse=5), "fp64"),  # 32 x 16, 16 segments of 8 levels
    ((128, 64, 200), dict(n_levels=3, nu_coarse=3), "fp64"),   # 16 segments of 13 levels (ragged)
    ((64, 64, 96), dict(n_levels=3, nu_coarse=2), "fp64"),     # 8 segments of 12 levels
    ((64, 64, 256), dict(n_levels=3, nu_coarse=1), "fp64"),    # 16 segments of 16 levels
    ((64, 32, 128), dict(n_levels=3, nu_coarse=5), "fp32"),    # one tile row; the FP32 coarsest level
])
def test_coarse_sweep_pairs_are_bitwise(ell, orc, shape, mg, precision):
    """Each coarsest-level sweep pair in one launch (k_coarse_pair: colour 0
    on the tile and its ring kept in LDS, then colour 1 on the tile) gives
    the V-cycle of two half-sweep launches bitwise, and (FP64) the oracle's."""
    g = grid_for(orc, shape, **mg)
    r = np.random.default_rng(13).standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    out = []
    for paired in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_COARSE_PAIR, paired)
        try:
            G = gpu_grid(ell, g, precision)
        finally:
            ell.set_tuning(ell.ELL_TUNE_COARSE_PAIR, 1)
        assert G.features["coarse_pair"] == bool(paired), G.features
        out.append(host(G.vcycle(dev(r))))
        G.close()
    assert np.array_equal(out[0], out[1])
    if precision == "fp64":
        assert rel(out[0], orc.vcycle(g, r)) <= 1e-11


@pytest.mark.parametrize("flexible", [False, True])
@pytest.mark.parametrize("nx,ny,nz,levels", [(64, 16, 32, 3), (68, 12, 100, 2), (136, 8, 40, 2),
                                           (64, 64, 48, 4)])
def test_fused_prolongation_equals_prolongation_pass(ell, orc, nx, ny, nz, levels, flexible):
    """With either beta, the finest coarse correction applied inside the
    first post-smoothing sweep (and <r, z>, with the flexible beta also
    <z, q>, of both colours formed by the last) gives the iterates of the
    prolongation pass: the same iteration count,
    solutions within 1e-10, the same state at an iteration limit, and the
    oracle's solution.  (136, 8) has partial tiles, nz = 100 eight ragged
    k-segments."""
    h = 1.0 / nx
    dz = I.dz_quadratic(nz, 1.0 / 50.0)
    p = I.Problem("fused_prolong", nx, ny, nz, h, h, dz, I.lambda2_perturbed(h, dz, 0.3, 26), 1e-2,
                  I.rhs_normal(nx, ny, dz, 25), n_levels=levels)
    res = []
    for fused in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_FUSED_PROLONG, fused)
        try:
            G = ell.Grid.from_problem(p)
        finally:
            ell.set_tuning(ell.ELL_TUNE_FUSED_PROLONG, 1)
        assert G.features["fused_prolong"] == bool(fused)
        u, st = G.pcg_solve(dev(p.f), rtol=1e-8, flexible=flexible)
        assert st.status == 0
        ul, stl = G.pcg_solve(dev(p.f), rtol=1e-14, maxiter=3, flexible=flexible)
        assert stl.status == ell.ELL_NOT_CONVERGED and stl.iters == 3
        res.append((host(u), st, host(ul), stl))
    (u1, s1, l1, t1), (u0, s0, l0, t0) = res
    assert s1.iters == s0.iters
    assert rel(u1, u0) <= 1e-10 and rel(l1, l0) <= 1e-10
    # the recurrence residual r_k = r_0 - sum alpha_i q_i after 3 steps lies
    # between 1e-3 and 0.07 of ||r0|| here: the fused dots sum in another order,
    # and rounding-size differences of alpha and beta reach r_k in proportion
    # to ||r0||, not to ||r_k||
    assert abs(t1.r_norm - t0.r_norm) <= 1e-9 * t0.r0_norm
    g = orc.Grid.from_problem(p)
    check_solve(orc, g, p.f, u1, s1, 1e-8, flexible=flexible)


@pytest.mark.parametrize("nx,ny,nz,levels", [(64, 16, 32, 3), (68, 12, 100, 2), (136, 36, 40, 2),
                                           (2, 8, 12, 2)])
def test_tiled_solve_ends_equal_column_kernels(ell, orc, nx, ny, nz, levels):
    """A solve's start (us = u0, r = V f - A u0 from a nonzero u0) and end (u =
    us + alpha p written plane-major, the true residual) on the operator
    step's LDS tiles give the column kernels' values: the same iterates
    bitwise at a fixed iteration count (CG and stand-alone multigrid), the
    norms up to summation order, and the oracle's norms of r0, V f and the
    true residual.  (68, 12) and (136, 36) have partial tiles in both
    directions, nz = 100 four 25-level segments, (2, 8) one-cell-wide tiles
    whose left and right neighbours are one cell."""
    h = 1.0 / nx
    dz = I.dz_quadratic(nz, 1.0 / 50.0)
    p = I.Problem("tiled_ends", nx, ny, nz, h, h, dz, I.lambda2_perturbed(h, dz, 0.3, 28), 1e-2,
                  I.rhs_normal(nx, ny, dz, 27), n_levels=levels)
    g = orc.Grid.from_problem(p)
    V = orc.level_coeffs(g)[0]
    b = V[:, None, None] * p.f
    bn = float(np.linalg.norm(b))
    # a random start scaled so that ||A u0|| = ||V f||
    u0 = np.random.default_rng(29).standard_normal(p.f.shape)
    u0 *= bn / np.linalg.norm(orc.apply(g, u0))
    res = []
    for tiled in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_TILED_ENDS, tiled)
        try:
            G = ell.Grid.from_problem(p)
        finally:
            ell.set_tuning(ell.ELL_TUNE_TILED_ENDS, 1)
        assert G.features["tiled_ends"] == bool(tiled)
        ul, stl = G.pcg_solve(dev(p.f), u=dev(u0), rtol=1e-14, maxiter=3)
        assert stl.status == ell.ELL_NOT_CONVERGED and stl.iters == 3
        um, stm = G.mg_solve(dev(p.f), u=dev(u0), rtol=1e-14, maxiter=2)
        assert stm.iters == 2
        u, st = G.pcg_solve(dev(p.f), u=dev(u0), rtol=1e-8)
        assert st.status == 0
        res.append((host(ul), stl, host(um), stm, host(u), st))
    (l1, t1, m1, n1, u1, s1), (l0, t0, m0, n0, u0c, s0) = res
    np.testing.assert_array_equal(l1, l0)
    np.testing.assert_array_equal(m1, m0)
    assert s1.iters == s0.iters
    assert rel(u1, u0c) <= 1e-12
    for sa, sb in ((t1, t0), (n1, n0), (s1, s0)):
        for k in ("r0_norm", "b_norm", "true_r_norm"):
            assert abs(getattr(sa, k) / getattr(sb, k) - 1) <= 1e-12, (k, getattr(sa, k), getattr(sb, k))
    assert abs(t1.b_norm / bn - 1) <= 1e-13

    def agree(gpu_norm, uu):
        # two FP64 evaluations of ||V f - A u||, each cell's terms in any
        # order (16 eps || |A| |u| + |V f| ||) and the sum of squares in any
        # order (n eps of the norm)
        eps = np.finfo(float).eps
        rn = np.linalg.norm(orc.residual(g, b, uu))
        tol = 16 * eps * np.linalg.norm(orc.apply_abs(g, np.abs(uu)) + np.abs(b)) + b.size * eps * rn
        return abs(gpu_norm - rn) <= tol

    assert agree(t1.r0_norm, u0)
    for uu, stt in ((l1, t1), (m1, n1), (u1, s1)):
        assert agree(stt.true_r_norm, uu)
    check_solve(orc, g, p.f, u1, s1, 1e-8, u0=u0)


@pytest.mark.parametrize("flexible", [False, True])
def test_deferred_updates_at_every_iteration_count(ell, orc, flexible):
    """The solution updates ride on the operator steps two at a time (odd
    steps from the third on) and the end of a solve applies what is pending
    (one update after an odd iteration count, two after an even one, through
    three rotating direction buffers): CG stopped after 1..6 iterations and
    stand-alone multigrid after 1..5 return the oracle's iterate."""
    p = I.graded_problem("defer", 64, 24, 1e-2, 41, 42)
    G = ell.Grid.from_problem(p)
    g = orc.Grid.from_problem(p)
    for k in range(1, 7):
        u, st = G.pcg_solve(dev(p.f), rtol=1e-15, maxiter=k, flexible=flexible)
        ur, sr = orc.pcg(g, p.f, rtol=1e-15, maxiter=k, flexible=flexible)
        assert st.iters == k and sr["iters"] == k
        assert rel(host(u), ur) <= 1e-10, k
    for k in range(1, 6):
        u, st = G.mg_solve(dev(p.f), rtol=1e-15, maxiter=k)
        ur, sr = orc.mg_solve(g, p.f, rtol=1e-15, maxiter=k)
        assert st.iters == k and sr["iters"] == k
        assert rel(host(u), ur) <= 1e-10, k


def test_solve_edge_cases(ell, orc):
    p = I.graded_problem("edge", 32, 8, 1e-2, 1, 2)
    G = ell.Grid.from_problem(p)
    g = orc.Grid.from_problem(p)
    # zero right-hand side: no iterations, u stays zero
    u, st = G.pcg_solve(torch.zeros(p.f.shape, dtype=torch.float64, device="cuda"))
    assert st.iters == 0 and st.status == 0 and not host(u).any()
    # maxiter reached: NOT_CONVERGED with the same iterate as the oracle
    u, st = G.pcg_solve(dev(p.f), rtol=1e-14, maxiter=2)
    u_ref, st_ref = orc.pcg(g, p.f, rtol=1e-14, maxiter=2)
    assert st.status == ell.ELL_NOT_CONVERGED and st.iters == 2 and st_ref["status"] == 1
    assert rel(host(u), u_ref) <= 1e-10
    # warm start relative to ||b||: a converged u needs no further iteration
    u, st = G.pcg_solve(dev(p.f), rtol=1e-8, rel_to_rhs=True)
    u2, st2 = G.pcg_solve(dev(p.f), u=u.clone(), rtol=1e-8, rel_to_rhs=True)
    assert st2.iters == 0
    # non-finite input is reported, not returned as a solution
    f = p.f.copy()
    f[3, 2, 1] = np.nan
    with pytest.raises(ell.EllError) as ei:
        G.pcg_solve(dev(f))
    assert ei.value.code == ell.ELL_ERR_NUMERIC
    # polling granularity does not change the result
    ua, sa = G.pcg_solve(dev(p.f), poll_every=1)
    ub, sb = G.pcg_solve(dev(p.f), poll_every=16)
    assert sa.iters == sb.iters
    np.testing.assert_array_equal(host(ua), host(ub))


# Shapes for the CG operator step: partial tiles in x and y (tiles are 64 x 16
# plane-major columns), uneven k-segments (nz = 70: four segments of 18, 18,
# 18, 16 levels), the smallest periodic grid (2 x 2) and a one-tile-wide one.
# The iteration counts stop each solve while its residual is still far above
# rounding (the 2 x 2 and 4 x 6 grids converge within a few iterations).
TILE_SHAPES = [((130, 38, 7), 6), ((34, 10, 33), 6), ((2, 2, 3), 2), ((4, 6, 70), 3),
               ((66, 18, 64), 6), ((64, 16, 5), 6)]


@pytest.mark.parametrize("shape,K", TILE_SHAPES)
def test_operator_step_tiles_fixed_iterations(ell, orc, shape, K):
    """K CG iterations (none converges) match the oracle's K, on the LDS-tiled
    operator step and on the column-walking one."""
    g = small_grid(orc, *shape, seed=5 + sum(shape), graded=False)
    f = np.random.default_rng(3).standard_normal(g.shape)
    f -= f.mean()
    u_ref, st_ref = orc.pcg(g, f, rtol=1e-30, maxiter=K)
    got = {}
    for tile in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_APPLY_TILE, tile)
        try:
            G = gpu_grid(ell, g)
        finally:
            ell.set_tuning(ell.ELL_TUNE_APPLY_TILE, 1)
        u, st = G.pcg_solve(dev(f), rtol=1e-30, maxiter=K)
        assert st.iters == st_ref["iters"] == K and st.status == ell.ELL_NOT_CONVERGED
        got[tile] = host(u)
        assert rel(got[tile], u_ref) <= 1e-12, (tile, rel(got[tile], u_ref))
        assert abs(st.r_norm / st_ref["r_norm"] - 1) <= 1e-9
    assert rel(got[1], got[0]) <= 1e-13


def test_autotuned_schedule_is_recorded_and_solves_match(ell, orc):
    """The autotuner returns a valid schedule for the shape, grids created
    afterwards use it, and a solve under it matches the oracle like any other
    (a schedule changes how the path runs, not what it computes)."""
    p = I.graded_problem("tune", 64, 64, 1e-2, 21, 22, n_levels=4, nu_coarse=5)
    kw = dict(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, omega2=p.omega2, dz=p.dz,
              lambda2=p.lambda2, n_levels=p.n_levels, nu_coarse=p.nu_coarse)
    try:
        best = ell.autotune(iters=3, **kw)
        assert best["ms_per_iter"] > 0 and best["smooth_nseg"][0] in (4, 8)
        assert len(best["smooth_nseg"]) == 4 and best["apply_nseg"] in (1, 2, 4)
        assert all(s in (4, 8, 16) for s in best["smooth_nseg"])
        assert {k: v for k, v in ell.schedule_get(**kw).items()} == best
        G = ell.Grid.from_problem(p)
        u, st = G.pcg_solve(dev(p.f), rtol=p.rtol)
        assert st.status == 0
        check_solve(orc, orc.Grid.from_problem(p), p.f, host(u), st, p.rtol)
        # explicitly chosen schedules compute the same five iterations
        ref, _ = G.pcg_solve(dev(p.f), rtol=1e-30, maxiter=5)
        ref = host(ref)
        for sch in (dict(apply_tile=0, apply_nseg=4, smooth_nseg=[4, 16, 16, 16]),
                    dict(apply_tile=1, apply_nseg=1, smooth_nseg=[4, 8, 8, 4])):
            ell.schedule_set(sch, **kw)
            u2, st2 = ell.Grid.from_problem(p).pcg_solve(dev(p.f), rtol=1e-30, maxiter=5)
            assert st2.iters == 5 and rel(host(u2), ref) <= 1e-12
    finally:
        ell.schedule_set(None, **kw)


def test_one_level_line_relaxation_cg_matches_oracle(ell, orc):
    """CG preconditioned by one block red/black SSOR sweep of vertical line
    relaxation (the paper's one-level solver, Table 2): same iterates as the
    oracle and the same iteration count as its classic-beta variant."""
    p = I.graded_problem("onelevel", 64, 32, 1e-2, 41, 42, n_levels=1, nu_coarse=0)
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p)
    assert G.levels == 1
    u, st = G.pcg_solve(dev(p.f), rtol=p.rtol)
    assert st.status == 0
    check_solve(orc, g, p.f, host(u), st, p.rtol)
    u2, st2 = G.pcg_solve(dev(p.f), rtol=p.rtol, flexible=False)
    assert abs(st2.iters - st.iters) <= 1


@pytest.mark.parametrize("name,kw", [
    ("config0", None),
    ("mg_graded64_L4", dict(nx=64, nz=32, n_levels=4, nu_coarse=5)),
    ("mg_graded96", dict(nx=96, nz=24)),
])
def test_standalone_multigrid_matches_oracle(ell, orc, name, kw):
    """Stand-alone multigrid (repeated V-cycles): four iterations equal the
    oracle's four, and the converged solve stops with it."""
    if kw is None:
        p = I.config0()
    else:
        kw = dict(kw)
        p = I.graded_problem(name, kw.pop("nx"), kw.pop("nz"), 1e-2, 51, 52, **kw)
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p)
    u, st = G.mg_solve(dev(p.f), rtol=1e-30, maxiter=4)
    u_ref, st_ref = orc.mg_solve(g, p.f, rtol=1e-30, maxiter=4)
    assert st.iters == st_ref["iters"] == 4 and st.status == ell.ELL_NOT_CONVERGED
    assert rel(host(u), u_ref) <= 1e-10
    assert abs(st.r_norm / st_ref["r_norm"] - 1) <= 1e-6
    u, st = G.mg_solve(dev(p.f), rtol=p.rtol)
    u_ref, st_ref = orc.mg_solve(g, p.f, rtol=p.rtol)
    assert st.status == 0 and abs(st.iters - st_ref["iters"]) <= 1, (st.iters, st_ref["iters"])
    if st.iters == st_ref["iters"]:
        assert rel(host(u), u_ref) <= 1e-10


def test_single_column_solve(ell, orc):
    g = small_grid(orc, 1, 1, 40, seed=2, graded=False)
    G = gpu_grid(ell, g)
    f = np.random.default_rng(9).standard_normal(g.shape)
    u, st = G.pcg_solve(dev(f), rtol=1e-12)
    u_ref, st_ref = orc.pcg(g, f, rtol=1e-12)
    assert st.iters == st_ref["iters"] == 1
    assert rel(host(u), u_ref) <= 1e-12


def test_invalid_arguments(ell):
    with pytest.raises(ell.EllError):
        ell.Grid(33, 32, 4, 0.1, 0.1, 1e-2, np.ones(4), np.ones(4))
    G = ell.Grid(8, 8, 4, 0.1, 0.1, 1e-2, np.ones(4), np.ones(4))
    x = torch.zeros((4, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ell.EllError):
        G.apply_A(x, x)
    with pytest.raises(ell.EllError):
        G.level_smooth(5, 0, G.level_empty(0), G.level_empty(0))
