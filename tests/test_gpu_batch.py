"""Batch engine: grouped launches over uneven grids with continuous
admission.  Every result must equal the same solve alone (bitwise: each grid
keeps its own deterministic reductions and the same kernels) and match the
oracle like a single-grid solve."""
import time

import numpy as np
import pytest
import torch

from paper_1307_2036_amd import inputs as I
from solve_parity import check_solve

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problems():
    # uneven sizes and depths: 64 (7 levels), 96 (5), 128 (8), 32 (6)
    return [I.graded_problem("b0", 64, 32, 1e-2, 31, 32),
            I.graded_problem("b1", 96, 24, 3e-2, 33, 34),
            I.graded_problem("b2", 128, 16, 1e-3, 35, 36),
            I.graded_problem("b3", 32, 40, 1e-1, 37, 38),
            I.graded_problem("b4", 64, 24, 5e-2, 39, 40, n_levels=4, nu_coarse=5)]


@pytest.fixture(scope="module")
def E():
    from paper_1307_2036_amd import ell
    return ell


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_alone_equals_in_mix_and_oracle(E, orc, precision):
    ps = problems()
    B = E.Batch(8 << 30)
    grids = [B.grid(p, precision=precision) for p in ps]
    fs = [dev(p.f) for p in ps]
    # the mix: all five together
    us = [torch.zeros_like(f) for f in fs]
    st_mix = B.wait(B.submit(grids, fs, us))
    mix = [host(u) for u in us]
    # each alone
    for i, (g, f) in enumerate(zip(grids, fs)):
        u1 = torch.zeros_like(f)
        st1 = B.wait(B.submit([g], [f], [u1]))
        assert st1[0].iters == st_mix[i].iters
        np.testing.assert_array_equal(host(u1), mix[i])
    # against the oracle (FP64 path; the mixed path as in the mixed-precision tests)
    for i, p in enumerate(ps):
        assert st_mix[i].status == 0
        g = orc.Grid.from_problem(p)
        if precision == "fp64":
            check_solve(orc, g, p.f, mix[i], st_mix[i], p.rtol)
        else:
            u64, s64 = orc.pcg(g, p.f, rtol=p.rtol)
            assert st_mix[i].iters <= s64["iters"] + 2
            assert np.linalg.norm(mix[i] - u64) <= 1e-4 * np.linalg.norm(u64)
    B.close()


def test_batch_fp32_validation_mode(E, orc):
    """The FP32 preconditioner in the batch, validation mode: every instance of
    the uneven mix solved together to rtol 1e-12 lies within 1e-8 of the FP64
    oracle's tight solution (the precision of the preconditioner changes the
    iterates, not the discrete solution)."""
    ps = problems()
    B = E.Batch(8 << 30)
    grids = [B.grid(p, precision="fp32") for p in ps]
    fs = [dev(p.f) for p in ps]
    us = [torch.zeros_like(f) for f in fs]
    st = B.wait(B.submit(grids, fs, us, rtol=1e-12, maxiter=400))
    for p, u, s in zip(ps, us, st):
        assert s.status == 0, (p.name, s)
        u_ref, s_ref = orc.pcg(orc.Grid.from_problem(p), p.f, rtol=1e-12, maxiter=400)
        err = float(np.linalg.norm(host(u) - u_ref) / np.linalg.norm(u_ref))
        print(p.name, "iters", s.iters, s_ref["iters"], "rel", err)
        assert err <= 1e-8, (p.name, err)
    B.close()


def test_batch_matches_single_grid_path(E, orc):
    """The batch (4- or 8-segment coarse levels, grouped kernels) and the
    single-grid path solve the same problem to the same iterates."""
    p = problems()[1]
    B = E.Batch(4 << 30)
    g = B.grid(p)
    f = dev(p.f)
    u = torch.zeros_like(f)
    st = B.wait(B.submit([g], [f], [u]))[0]
    G = E.Grid.from_problem(p)
    u2, st2 = G.pcg_solve(f, rtol=p.rtol)
    assert st.iters == st2.iters
    assert np.linalg.norm(host(u) - host(u2)) <= 1e-12 * np.linalg.norm(host(u2))
    B.close()


def test_deferred_updates_in_batch(E, orc):
    """Batched solves stopped after 1..6 iterations (the end of each applying
    the one or two solution updates still pending) return the oracle's
    iterate."""
    ps = problems()[:2]
    B = E.Batch(4 << 30)
    grids = [B.grid(p) for p in ps]
    gs = [orc.Grid.from_problem(p) for p in ps]
    for k in range(1, 7):
        fs = [dev(p.f) for p in ps]
        us = [torch.zeros_like(f) for f in fs]
        st = B.wait(B.submit(grids, fs, us, rtol=1e-15, maxiter=k))
        for p, g, u, s in zip(ps, gs, us, st):
            ur, sr = orc.pcg(g, p.f, rtol=1e-15, maxiter=k)
            assert s.iters == k and sr["iters"] == k
            assert np.linalg.norm(host(u) - ur) <= 1e-10 * np.linalg.norm(ur), k
    B.close()


def test_continuous_admission_and_warm_start(E, orc):
    """A ticket submitted while another runs joins the running iterations; two
    requests on one grid run one after the other (the second warm-starts)."""
    ps = problems()
    B = E.Batch(8 << 30)
    grids = [B.grid(p) for p in ps]
    fs = [dev(p.f) for p in ps]
    us = [torch.zeros_like(f) for f in fs]
    t1 = B.submit(grids[:3], fs[:3], us[:3], rel_to_rhs=True)
    u_late = torch.zeros_like(fs[3])
    t2 = B.submit([grids[3]], [fs[3]], [u_late], rel_to_rhs=True)
    # same grid again: queued behind t1's request on grid 0, warm start from its result
    t3 = B.submit([grids[0]], [fs[0]], [us[0]], rel_to_rhs=True)
    s1, s2, s3 = B.wait(t1), B.wait(t2), B.wait(t3)
    assert all(s.status == 0 for s in s1 + s2 + s3)
    assert s3[0].iters == 0  # already converged relative to ||b||
    g = orc.Grid.from_problem(ps[3])
    u_ref, st_ref = orc.pcg(g, ps[3].f, rtol=ps[3].rtol, rel_to_rhs=True)
    assert np.linalg.norm(host(u_late) - u_ref) <= 1e-6 * np.linalg.norm(u_ref)
    B.close()


def test_budget_and_validation(E):
    p = problems()[0]
    need = E.grid_bytes(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, omega2=p.omega2, dz=p.dz,
                        lambda2=p.lambda2)
    B = E.Batch(int(1.5 * need))
    g = B.grid(p)
    with pytest.raises(E.EllError) as ei:
        B.grid(p)
    assert ei.value.code == E.ELL_ERR_BUDGET
    used = B.bytes_in_use()
    g.close()
    assert B.bytes_in_use() < used
    g2 = B.grid(p)  # fits again after the release
    with pytest.raises(E.EllError):
        B.grid(p, precision="fp32")  # mixed precision classes in one batch
    B.close()
    B2 = E.Batch(1 << 30)
    with pytest.raises(E.EllError):
        B2.grid(p, rho=0.9)
    g3 = B2.grid(p)
    with pytest.raises(E.EllError):
        B2.grid(p, nu_post=2)  # one smoothing schedule per batch
    g3.close()
    B2.close()


def test_poll_pending_then_done(E):
    p = problems()[2]
    B = E.Batch(4 << 30)
    g = B.grid(p)
    f = dev(p.f)
    u = torch.zeros_like(f)
    t = B.submit([g], [f], [u])
    deadline = time.time() + 60
    res = None
    while res is None and time.time() < deadline:
        res = B.poll(t)
        time.sleep(0.001)
    assert res is not None and res[0].status == 0
    B.wait(t)
    B.close()


def test_graph_replays_equal_direct_launches(E):
    """Grouped steps replayed from captured graphs give the same bits as direct
    launches.  Each batch replays its graphs many times (two steps per poll,
    a new capture whenever a grid converges and leaves; the second batch polls
    every step, so each new stage table first launches directly and is
    captured when it runs again), with other GPU work and synchronisations
    between the solves; every result is compared."""
    ps = problems()
    res = {}
    for graph in (0, 1):
        E.set_tuning(E.ELL_TUNE_BATCH_GRAPH, graph)
        try:
            B = E.Batch(8 << 30)
        finally:
            E.set_tuning(E.ELL_TUNE_BATCH_GRAPH, 1)
        grids = [B.grid(p, precision="fp32") for p in ps]
        out = []
        for rep in range(3):
            fs = [dev(p.f * (1.0 + 0.5 * rep)) for p in ps]
            us = [torch.zeros_like(f) for f in fs]
            noise = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
            st = B.wait(B.submit(grids, fs, us, poll_every=1 if rep == 1 else 2))
            torch.cuda.synchronize()
            assert torch.isfinite(noise)
            out.append(([host(u) for u in us], [s.iters for s in st]))
        res[graph] = out
        B.close()
    for (u0, i0), (u1, i1) in zip(res[0], res[1]):
        assert i0 == i1
        for a, b in zip(u0, u1):
            np.testing.assert_array_equal(a, b)


def test_failures_stay_with_their_request(E):
    """A request whose right-hand side holds a NaN ends with a numeric error,
    a request that hits its iteration limit ends not converged, and the other
    requests of the same grouped launches finish exactly as they do alone."""
    ps = problems()[:3]
    B = E.Batch(8 << 30)
    grids = [B.grid(p, precision="fp32") for p in ps]
    fs = [dev(p.f) for p in ps]
    bad = fs[1].clone()
    bad[2, 3, 4] = float("nan")
    us = [torch.zeros_like(f) for f in fs]
    t_ok = B.submit([grids[0]], [fs[0]], [us[0]])
    t_bad = B.submit([grids[1]], [bad], [us[1]])
    t_lim = B.submit([grids[2]], [fs[2]], [us[2]], rtol=1e-14, maxiter=2)
    st_ok = B.wait(t_ok)
    st_bad = B.wait(t_bad, check=False)
    st_lim = B.wait(t_lim, check=False)
    assert st_ok[0].status == E.ELL_OK
    assert st_bad[0].status == E.ELL_ERR_NUMERIC
    assert st_lim[0].status == E.ELL_NOT_CONVERGED and st_lim[0].iters == 2
    u_alone = torch.zeros_like(fs[0])
    st_alone = B.wait(B.submit([grids[0]], [fs[0]], [u_alone]))
    assert st_alone[0].iters == st_ok[0].iters
    np.testing.assert_array_equal(host(u_alone), host(us[0]))
    B.close()


@pytest.mark.slow
def test_config3_batch_at_full_size(E, orc):
    """The 64 seeded uneven instances of the batched workload, solved together
    exactly as the benchmark does (grouped launches, FP32 preconditioner, 1e-5):
    every solve converges within the FP64 oracle's iteration count + 2 on the
    sampled instances, and its solution lies within 1e-4 of the oracle's."""
    ps = I.config3_instances(64)
    B = E.Batch(200 << 30)
    grids = [B.grid(p, precision="fp32") for p in ps]
    fs = [dev(p.f) for p in ps]
    us = [torch.zeros_like(f) for f in fs]
    st = B.wait(B.submit(grids, fs, us, rtol=1e-5, poll_every=4))
    assert all(s.status == 0 for s in st)
    assert all(1 <= s.iters <= 20 for s in st)
    # sampled instances: the two largest and four by seed
    sizes = [p.n for p in ps]
    picks = sorted(set([int(np.argmax(sizes)), int(np.argsort(sizes)[-2])] +
                       list(np.random.default_rng(3).choice(64, 4, replace=False))))
    for i in picks:
        g = orc.Grid.from_problem(ps[i])
        u_ref, st_ref = orc.pcg(g, ps[i].f, rtol=ps[i].rtol)
        assert st[i].iters <= st_ref["iters"] + 2, (i, st[i].iters, st_ref["iters"])
        u = host(us[i])
        assert np.linalg.norm(u - u_ref) <= 1e-4 * np.linalg.norm(u_ref), i
    B.close()


@pytest.mark.slow
def test_config3_batch_fp32_validation_mode(E, orc):
    """The 64 instances of the batched workload together with the FP32
    preconditioner to rtol 1e-12: the two largest and four sampled instances
    lie within 1e-8 of the FP64 oracle's tight solutions."""
    ps = I.config3_instances(64)
    B = E.Batch(200 << 30)
    grids = [B.grid(p, precision="fp32") for p in ps]
    fs = [dev(p.f) for p in ps]
    us = [torch.zeros_like(f) for f in fs]
    st = B.wait(B.submit(grids, fs, us, rtol=1e-12, maxiter=400, poll_every=4))
    assert all(s.status == 0 for s in st)
    sizes = [p.n for p in ps]
    picks = sorted(set([int(np.argmax(sizes)), int(np.argsort(sizes)[-2])] +
                       list(np.random.default_rng(3).choice(64, 4, replace=False))))
    for i in picks:
        u_ref, s_ref = orc.pcg(orc.Grid.from_problem(ps[i]), ps[i].f, rtol=1e-12, maxiter=400)
        err = float(np.linalg.norm(host(us[i]) - u_ref) / np.linalg.norm(u_ref))
        print(ps[i].name, "iters", st[i].iters, s_ref["iters"], "rel", err)
        assert err <= 1e-8, (i, err)
    B.close()


@pytest.mark.parametrize("precision,flexible", [("fp32", True), ("fp64", False), ("fp64", True)])
def test_fused_dots_and_tiles_in_batch(E, precision, flexible):
    """The batch's tiled finest-level half-sweeps with the fused CG dots and the
    fused residual update give the iterates of the batch without them (column
    kernels, separate passes) up to the summation order; (96, 24) has a partial
    tile and (32, 40) one tile per row pair."""
    ps = problems()
    res = []
    for on in (1, 0):
        E.set_tuning(E.ELL_TUNE_FUSED_DOT, on)
        E.set_tuning(E.ELL_TUNE_SMOOTH_TILE, on)
        E.set_tuning(E.ELL_TUNE_FUSED_UPDATE, on)
        try:
            B = E.Batch(8 << 30)
            grids = [B.grid(p, precision=precision) for p in ps]
        finally:
            E.set_tuning(E.ELL_TUNE_FUSED_DOT, 1)
            E.set_tuning(E.ELL_TUNE_SMOOTH_TILE, 1)
            E.set_tuning(E.ELL_TUNE_FUSED_UPDATE, 1)
        fs = [dev(p.f) for p in ps]
        us = [torch.zeros_like(f) for f in fs]
        st = B.wait(B.submit(grids, fs, us, rtol=1e-8, flexible=flexible))
        res.append(([host(u) for u in us], [s.iters for s in st]))
        B.close()
    (u1, i1), (u0, i0) = res
    assert i1 == i0
    for a, b in zip(u1, u0):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("flexible", [True, False])
def test_mixed_fused_prolongation_in_batch_is_bitwise(E, flexible):
    """The mixed-precision batch's finest prolongation applied inside the first
    FP64 colour-1 post-smoothing sweep (FP32 colour-0 values and coarse
    correction staged, the correction formed in FP32 and added in FP64) gives
    the iterates of the batch with the prolongation pass, bitwise, with the
    fused dots of either beta; the grids differ in size, depth and segments."""
    ps = problems()
    res = []
    for on in (1, 0):
        E.set_tuning(E.ELL_TUNE_FUSED_PROLONG, on)
        try:
            B = E.Batch(8 << 30)
            grids = [B.grid(p, precision="fp32") for p in ps]
        finally:
            E.set_tuning(E.ELL_TUNE_FUSED_PROLONG, 1)
        fs = [dev(p.f) for p in ps]
        us = [torch.zeros_like(f) for f in fs]
        st = B.wait(B.submit(grids, fs, us, rtol=1e-8, flexible=flexible))
        assert all(s.status == 0 for s in st)
        res.append(([host(u) for u in us], [s.iters for s in st]))
        B.close()
    (u1, i1), (u0, i0) = res
    assert i1 == i0
    for a, b in zip(u1, u0):
        np.testing.assert_array_equal(a, b)
