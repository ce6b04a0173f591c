"""GPU parity of horizontally varying vertical coefficients (a 3D lambda^2
field: every column its own vertical faces and Thomas factors; coarse faces
are the sums of the children's) against the oracle, through the C ABI.

Operator (Sec. 3.1), both colours of line relaxation on every level (Sec. 4.2
eq. BlockRBSOR, Appendix B Thomas algorithm per column), residual plus
restriction, one V-cycle (Sec. 4.3), and whole solves (Appendix B, Alg. PCG;
stand-alone multigrid) at equal iteration counts, also at 512 x 512 x 128."""
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def zeros(shape):
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def pair(ell, orc, nx, ny, nz, seed=1, sigma=0.8, graded=True, **mg):
    """Oracle grid with per-column faces and the GPU grid of the same field."""
    g = small_grid(orc, nx, ny, nz, graded=graded, seed=seed, **mg)
    lam3 = I.lambda2_3d(nx, ny, g.lambda2, sigma, seed + 100)
    g.tz3 = orc.tz3_from_lambda2(nx, ny, nz, g.hx, g.hy, g.omega2, g.dz, lam3)
    G = ell.Grid(g.nx, g.ny, g.nz, g.hx, g.hy, g.omega2, g.dz, g.lambda2, g.n_levels, g.nu_pre, g.nu_post,
                 g.nu_coarse, g.rho, g.prolong, lambda2_3d=lam3)
    return g, G, lam3


SHAPES = [((64, 32, 24), 3), ((34, 10, 100), 1), ((68, 12, 100), 2), ((6, 1, 5), 1), ((1, 6, 4), 1),
          ((16, 8, 300), 2), ((32, 32, 16), 0)]


@pytest.mark.parametrize("shape,levels", SHAPES)
def test_varying_operator_and_levels_match_oracle(ell, orc, shape, levels):
    nx, ny, nz = shape
    g, G, _ = pair(ell, orc, nx, ny, nz, seed=nx + nz, n_levels=levels)
    f = G.features
    assert G.varying and not (f["tiled_smooth"] or f["fused_prolong"] or f["tiled_ends"] or f["coarse_prolong"])
    # the fused CG forms ride on the per-column sweep where it applies
    seg3 = nx > 1 and ny > 1 and nz <= 256 and G.levels >= 2
    assert f["fused_dots"] == seg3 and f["fused_update"] == seg3, (shape, f)
    rng = np.random.default_rng(nz)
    x = rng.standard_normal(g.shape)
    y = host(G.apply_A(dev(x)))
    assert np.all(np.abs(y - orc.apply(g, x)) <= 16 * EPS * orc.apply_abs(g, x))
    gl = g
    for lv in range(G.levels):
        # operator of the level (coarse faces summed from the children's)
        xl = rng.standard_normal(gl.shape)
        yl = zeros(gl.shape)
        ys = G.level_empty(lv)
        G.level_apply(lv, G.to_split(lv, dev(xl)), ys)
        yl = host(G.from_split(lv, ys, yl))
        assert np.all(np.abs(yl - orc.apply(gl, xl)) <= 16 * EPS * orc.apply_abs(gl, xl)), lv
        # red from zero, black, red again (rho = 1)
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
            # residual + restriction, general and after a colour-1 sweep
            u = rng.standard_normal(gl.shape)
            gc = gl.coarse()
            for bz in (False, True):
                uu = u
                if bz:
                    uu = orc.smooth_colour(gl, 1, b, u)
                bc = G.level_empty(lv + 1)
                G.level_resid_restrict(lv, bs, G.to_split(lv, dev(uu)), bc, black_zero=bz)
                got = host(G.from_split(lv + 1, bc, zeros(gc.shape)))
                ref = orc.restrict(gl, orc.residual(gl, b, uu))
                bound = 64 * EPS * orc.restrict(gl, orc.apply_abs(gl, uu) + np.abs(b))
                assert np.all(np.abs(got - ref) <= bound), (lv, bz)
            gl = gc


@pytest.mark.parametrize("shape,levels,rho", [((64, 32, 24), 3, 1.0), ((32, 16, 40), 0, 1.0),
                                              ((16, 16, 12), 2, 0.8), ((1, 1, 33), 1, 1.0)])
def test_varying_vcycle_matches_oracle(ell, orc, shape, levels, rho):
    nx, ny, nz = shape
    g, G, _ = pair(ell, orc, nx, ny, nz, seed=nx * ny + nz, n_levels=levels, rho=rho, nu_coarse=2)
    r = np.random.default_rng(4).standard_normal(g.shape) * (g.hx * g.hy * g.dz)[:, None, None]
    assert rel(host(G.vcycle(dev(r))), orc.vcycle(g, r)) <= 1e-11


@pytest.mark.parametrize("shape,levels", [((64, 64, 32), 0), ((96, 32, 64), 3), ((32, 32, 130), 0)])
def test_varying_solves_match_oracle(ell, orc, shape, levels):
    nx, ny, nz = shape
    p = I.paper_graded_problem(f"var{nx}", nx, ny, nz, 1e-2, 11 + nz, 12 + nz)
    p.n_levels = levels
    p.lambda2_3d = I.lambda2_3d(nx, ny, p.lambda2, 0.8, 13 + nz)
    g = orc.Grid.from_problem(p)
    assert g.tz3 is not None
    G = ell.Grid.from_problem(p)
    for flexible in (True, False):
        u, st = G.pcg_solve(dev(p.f), rtol=p.rtol, flexible=flexible)
        assert st.status == 0
        print(shape, flexible, check_solve(orc, g, p.f, host(u), st, p.rtol, flexible=flexible))
    u, st = G.mg_solve(dev(p.f), rtol=p.rtol)
    assert st.status == 0
    u_k, st_k = orc.mg_solve(g, p.f, rtol=0.0, maxiter=st.iters)
    assert rel(host(u), u_k) <= 1e-10


@pytest.mark.parametrize("shape,levels,precision", [((64, 32, 24), 3, "fp64"), ((96, 32, 64), 3, "fp64"),
                                                    ((68, 12, 100), 2, "fp64"), ((136, 24, 40), 0, "fp64"),
                                                    ((64, 64, 32), 0, "fp32"), ((96, 32, 64), 3, "fp32")])
def test_varying_fused_forms_equal_separate_passes(ell, orc, shape, levels, precision):
    """With per-column coefficients the CG residual update rides on the first
    pre-smoothing pair and the dots on the last post-smoothing pair
    (k_smooth_seg3's UPD and DOT forms): the same iteration counts and
    iterates within 1e-10 as the separate passes, for both betas in FP64 and
    the flexible one in mixed precision, the same state at an iteration limit,
    and (FP64) the oracle's solution.  (68, 12): eight ragged k-segments;
    (136, 24): a partial 64-column block."""
    nx, ny, nz = shape
    p = I.paper_graded_problem(f"varf{nx}", nx, ny, nz, 1e-2, 41 + nz, 42 + nz)
    p.n_levels = levels
    p.lambda2_3d = I.lambda2_3d(nx, ny, p.lambda2, 0.8, 43 + nz)
    betas = (True, False) if precision == "fp64" else (True,)
    res = {}
    for fused in (1, 0):
        ell.set_tuning(ell.ELL_TUNE_FUSED_DOT, fused)
        ell.set_tuning(ell.ELL_TUNE_FUSED_UPDATE, fused)
        try:
            G = ell.Grid.from_problem(p, precision=precision)
        finally:
            ell.set_tuning(ell.ELL_TUNE_FUSED_DOT, 1)
            ell.set_tuning(ell.ELL_TUNE_FUSED_UPDATE, 1)
        assert G.features["fused_dots"] == bool(fused) and G.features["fused_update"] == bool(fused)
        for flexible in betas:
            u, st = G.pcg_solve(dev(p.f), rtol=1e-8, flexible=flexible)
            assert st.status == 0
            ul, stl = G.pcg_solve(dev(p.f), rtol=1e-14, maxiter=3, flexible=flexible)
            assert stl.status == ell.ELL_NOT_CONVERGED and stl.iters == 3
            res[fused, flexible] = (host(u), st, host(ul), stl)
        G.close()
    for flexible in betas:
        (u1, s1, l1, t1), (u0, s0, l0, t0) = res[1, flexible], res[0, flexible]
        assert s1.iters == s0.iters
        assert rel(u1, u0) <= 1e-10 and rel(l1, l0) <= 1e-10
        assert abs(t1.r_norm / t0.r_norm - 1) <= 1e-8
        if precision == "fp64":
            check_solve(orc, orc.Grid.from_problem(p), p.f, u1, s1, 1e-8, flexible=flexible)


def colour_mask(nx, ny):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return (i + j) % 2


@pytest.mark.parametrize("shape,levels", [((64, 32, 24), 3), ((68, 12, 100), 2), ((6, 1, 5), 1),
                                          ((16, 8, 300), 2), ((40, 24, 200), 3)])
def test_varying_sweep_and_restriction_skip_poison(ell, orc, shape, levels):
    """Colour discipline with per-column coefficients (rho = 1): NaN in the
    old values of the colour being swept never reaches the output, which
    equals the sweep from zeroed own-colour values bitwise, on every level and
    for both colours (k_smooth_seg3; the column kernel on the one-wide grid
    and for 300 levels); the restriction right after a colour-1 sweep never
    reads colour 1 of the right-hand side (k_resid_restrict_bz with faces)."""
    nx, ny, nz = shape
    g, G, _ = pair(ell, orc, nx, ny, nz, seed=5 * nx + nz, n_levels=levels)
    rng = np.random.default_rng(3 * nx + nz)
    gl = g
    for lv in range(G.levels):
        mask = colour_mask(gl.nx, gl.ny)
        b = rng.standard_normal(gl.shape) * (gl.hx * gl.hy * gl.dz)[:, None, None]
        u = rng.standard_normal(gl.shape) * 1e-3
        bs = G.to_split(lv, dev(b))
        for c in (0, 1):
            own = np.broadcast_to(mask == c, gl.shape)
            out = []
            for start in (np.where(own, 0.0, u), np.where(own, np.nan, u)):
                us = G.to_split(lv, dev(start))
                G.level_smooth(lv, c, bs, us)
                out.append(host(G.from_split(lv, us, zeros(gl.shape))))
            assert np.all(np.isfinite(out[1])), (lv, c)
            np.testing.assert_array_equal(out[1], out[0])
        if lv + 1 < G.levels:
            gc = gl.coarse()
            black = np.broadcast_to(mask == 1, gl.shape)
            us = G.level_empty(lv)
            G.level_smooth(lv, 0, bs, us, zero_init=True)
            G.level_smooth(lv, 1, bs, us)
            res = []
            for bb in (b, np.where(black, np.nan, b)):
                bc = G.level_empty(lv + 1)
                G.level_resid_restrict(lv, G.to_split(lv, dev(bb)), us, bc, black_zero=True)
                res.append(host(G.from_split(lv + 1, bc, zeros(gc.shape))))
            assert np.all(np.isfinite(res[1])), lv
            np.testing.assert_array_equal(res[1], res[0])
            gl = gc


def test_horizontally_constant_field_equals_the_plain_grid(ell, orc):
    p = I.paper_graded_problem("const3d", 64, 32, 40, 1e-2, 5, 6)
    G0 = ell.Grid.from_problem(p)
    G3 = ell.Grid.from_problem(p, lambda2_3d=np.broadcast_to(p.lambda2[:, None, None], (40, 32, 64)))
    f = dev(p.f)
    u0, s0 = G0.pcg_solve(f, rtol=0.0, maxiter=6)
    u3, s3 = G3.pcg_solve(f, rtol=0.0, maxiter=6)
    assert s0.iters == s3.iters == 6
    assert rel(host(u3), host(u0)) <= 1e-12


def test_varying_grid_rejects_bad_input(ell, orc):
    p = I.paper_graded_problem("bad3d", 16, 16, 8, 1e-2, 5, 6)
    lam3 = I.lambda2_3d(16, 16, p.lambda2, 0.5, 7)
    with pytest.raises(ell.EllError) as e:
        ell.Grid.from_problem(p, precision="bf16coef", lambda2_3d=lam3)
    assert e.value.code == ell.ELL_ERR_INVALID
    bad = lam3.copy()
    bad[3, 2, 1] = 0.0
    with pytest.raises(ell.EllError) as e:
        ell.Grid.from_problem(p, lambda2_3d=bad)
    assert e.value.code == ell.ELL_ERR_INVALID


@pytest.mark.slow
def test_varying_fullsize_solve(ell, orc):
    """512 x 512 x 128, the graded lambda^2 profile of the benchmark solve modulated horizontally,
    four levels, five coarse sweeps: the iterates at the GPU's stopping count
    against the oracle's (printed beta)."""
    p = I.varying_problem()
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p)
    u, st = G.pcg_solve(dev(p.f), rtol=p.rtol, flexible=False)
    assert st.status == 0
    u_k, st_k = orc.pcg(g, p.f, rtol=0.0, maxiter=st.iters, flexible=False)
    err = rel(host(u), u_k)
    print("varying 512^2x128: iters", st.iters, "rel_l2", err)
    assert err <= 1e-10


VARYING_MIXED = [((64, 64, 32), 0), ((96, 32, 64), 3), ((32, 32, 130), 0), ((64, 32, 200), 2)]


def varying_problem_small(nx, ny, nz, levels):
    p = I.paper_graded_problem(f"varm{nx}", nx, ny, nz, 1e-2, 31 + nz, 32 + nz)
    p.n_levels = levels
    p.lambda2_3d = I.lambda2_3d(nx, ny, p.lambda2, 0.8, 33 + nz)
    return p


@pytest.mark.parametrize("shape,levels", VARYING_MIXED)
def test_varying_mixed_vcycle_and_tight_solve(ell, orc, shape, levels):
    """FP32 V-cycle with FP32 per-column fields (the FP64 finest post-smoothing
    also reads them): one V-cycle agrees with the oracle's FP64 one to FP32
    accuracy; solved to rtol 1e-12 the mixed solve reaches the oracle's tight
    solution to 1e-8; at 1e-5 it needs at most two iterations more than FP64."""
    nx, ny, nz = shape
    p = varying_problem_small(nx, ny, nz, levels)
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p, precision="fp32")
    assert G.varying
    r = p.f * (p.hx * p.hy * p.dz)[:, None, None]
    assert rel(host(G.vcycle(dev(r))), orc.vcycle(g, r)) <= 1e-5
    u_ref, _ = orc.pcg(g, p.f, rtol=1e-12, maxiter=400)
    u, st = G.pcg_solve(dev(p.f), rtol=1e-12, maxiter=400)
    assert st.status == 0, st
    err = rel(host(u), u_ref)
    print(shape, "tight iters", st.iters, "rel", err)
    assert err <= 1e-8
    G64 = ell.Grid.from_problem(p)
    _, s64 = G64.pcg_solve(dev(p.f), rtol=p.rtol)
    _, s32 = G.pcg_solve(dev(p.f), rtol=p.rtol)
    assert s32.status == 0 and s32.iters <= s64.iters + 2, (s32.iters, s64.iters)


def test_varying_mixed_levels_match_oracle(ell, orc):
    """FP32 levels of a varying grid: both colours of line relaxation and the
    restriction on every level against the oracle, to FP32 accuracy scaled by
    each column's largest value."""
    p = varying_problem_small(64, 32, 48, 3)
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p, precision="fp32")
    rng = np.random.default_rng(3)
    gl = g
    for lv in range(G.levels):
        b = rng.standard_normal(gl.shape) * (gl.hx * gl.hy * gl.dz)[:, None, None]
        bs = G.to_split(lv, dev(b))
        us = G.level_empty(lv)
        G.level_smooth(lv, 0, bs, us, zero_init=True)
        G.level_smooth(lv, 1, bs, us)
        ref = orc.smooth_colour(gl, 1, b, orc.smooth_colour(gl, 0, b, np.zeros(gl.shape)))
        got = host(G.from_split(lv, us, zeros(gl.shape)))
        scale = np.abs(ref).max(axis=0, keepdims=True)
        assert np.all(np.abs(got - ref) <= 1e-4 * scale), (lv, (np.abs(got - ref) / scale).max())
        if lv + 1 < G.levels:
            gl = gl.coarse()
