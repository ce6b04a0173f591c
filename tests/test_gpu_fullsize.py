"""Parity at the full production shape (512 x 512 x 128, graded, four levels,
five coarse sweeps) in the launch configuration the benchmark times: the
operator, one V-cycle and the whole solve against the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_1307_2036_amd import inputs as I

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def c1():
    from oracle import oracle as O
    from paper_1307_2036_amd import ell
    p = I.config1()
    return p, O.Grid.from_problem(p), ell.Grid.from_problem(p)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_fullsize_operator(orc, c1):
    p, g, G = c1
    x = I.random_field(p.nx, p.ny, p.nz, 5)
    y = host(G.apply_A(dev(x)))
    ref = orc.apply(g, x)
    assert np.all(np.abs(y - ref) <= 16 * EPS * orc.apply_abs(g, x))


def test_fullsize_vcycle(orc, c1):
    p, g, G = c1
    r = p.f * (p.hx * p.hy * p.dz)[:, None, None]
    z = host(G.vcycle(dev(r)))
    ref = orc.vcycle(g, r)
    print("vcycle rel", rel(z, ref))
    assert rel(z, ref) <= 1e-11


def test_fullsize_smoother_levels(orc, c1):
    """One half-sweep on every level of the hierarchy (both colours, from a
    non-zero start) against the oracle."""
    p, g, G = c1
    gl = g
    for lv in range(G.levels):
        rng = np.random.default_rng(lv)
        b = rng.standard_normal(gl.shape) * (gl.hx * gl.hy * gl.dz)[:, None, None]
        u0 = 0.009 + 1e-4 * rng.standard_normal(gl.shape)
        bs, us = G.to_split(lv, dev(b)), G.to_split(lv, dev(u0))
        G.level_smooth(lv, 0, bs, us)
        G.level_smooth(lv, 1, bs, us)
        got = host(G.from_split(lv, us, torch.zeros(gl.shape, dtype=torch.float64, device="cuda")))
        ref = orc.smooth_colour(gl, 1, b, orc.smooth_colour(gl, 0, b, u0))
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print("level", lv, "smoother max rel err", err)
        assert err <= 1e-13
        gl = gl.coarse()


def test_fullsize_solve(orc, c1):
    from solve_parity import check_solve
    p, g, G = c1
    u, st = G.pcg_solve(dev(p.f), rtol=p.rtol)
    assert st.status == 0
    info = check_solve(orc, g, p.f, host(u), st, p.rtol)
    print("solve parity", info)


def test_fullsize_solve_printed_beta(orc, c1):
    """The solve the benchmark times: the printed beta of Appendix B's PCG,
    which takes the fused finest prolongation (k_smooth_tile_pro) and the
    colour-0 sweep forming <r, z> of both colours (k_smooth_tile_dot3), against
    the oracle with the same beta at the full 512 x 512 x 128 size."""
    from solve_parity import check_solve
    p, g, G = c1
    assert G.features["fused_prolong"] and G.features["fused_dots"] and G.features["fused_update"]
    f = dev(p.f)
    u = torch.zeros_like(f)
    _, st = G.pcg_solve(f, u, rtol=p.rtol, maxiter=500, poll_every=8, flexible=False)
    assert st.status == 0
    info = check_solve(orc, g, p.f, host(u), st, p.rtol, flexible=False)
    print("printed-beta solve parity", info)


@pytest.mark.parametrize("levels,nu_coarse", [(5, 5), (0, 1)])
def test_fullsize_solve_other_depths(orc, levels, nu_coarse):
    """The same problem with four coarsenings (five levels, five coarsest
    sweeps; the other reading of the configuration's 'four coarsening
    levels') and at standard depth (ten levels, down to one column), printed
    beta, against the oracle."""
    from paper_1307_2036_amd import ell
    from solve_parity import check_solve
    p = I.config1(n_levels=levels, nu_coarse=nu_coarse)
    g = orc.Grid.from_problem(p)
    G = ell.Grid.from_problem(p)
    assert G.levels == (levels or 10) == orc.num_levels(g)
    f = dev(p.f)
    u = torch.zeros_like(f)
    _, st = G.pcg_solve(f, u, rtol=p.rtol, poll_every=8, flexible=False)
    assert st.status == 0
    info = check_solve(orc, g, p.f, host(u), st, p.rtol, flexible=False)
    print("levels", G.levels, "solve parity", info)
    G.close()
