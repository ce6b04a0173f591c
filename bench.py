"""Benchmark: FP64 multigrid-preconditioned CG on the 512 x 512 x 128 graded
production-shaped problem (four-level hierarchy, five coarse sweeps).

One step = one whole solve to a 1e-5 relative residual reduction from a zero
initial guess, with f resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s & unknowns·iter/s to 1e-5 rel. residual; HBM GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16coef"])
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--nu-coarse", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c1", choices=["c1", "c2", "batch", "serve", "robust"],
                    help="c1: the 512^2x128 solve (default); batch: 64 uneven solves in the "
                         "batch engine vs sequential FP64; serve: Poisson request stream")
    ap.add_argument("--autotune", action="store_true",
                    help="run the schedule autotuner on the workload's grid shape(s) before timing "
                         "(outside the timed region) and report the chosen schedule")
    ap.add_argument("--batch-graph", type=int, default=1, choices=[0, 1],
                    help="batch/serve: replay each grouped step from a captured HIP graph (1) "
                         "or launch its kernels directly (0)")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="arrival rate as a fraction of the measured closed-loop capacity")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain device copy of a 268 MB vector (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum seconds of oracle work in the CPU-baseline sample")
    return ap.parse_args()


def _desc_kw(p, precision):
    """Grid descriptor arguments of a seeded problem."""
    return dict(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, omega2=p.omega2, dz=p.dz,
                lambda2=p.lambda2, n_levels=p.n_levels, nu_pre=p.nu_pre, nu_post=p.nu_post,
                nu_coarse=p.nu_coarse, rho=p.rho, prolong=p.prolong, precision=precision)


def counter_traffic(precision: str):
    """HBM bytes per finest-level smoother launch from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, if it was taken on the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "smooth0_traffic.json")
    src = os.path.join(ROOT, "paper_1307_2036_amd", "csrc", "ell_kernels.hpp")
    if precision != "fp64" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("kernel_source_sha256_16") != cur:
        return None
    return rec["smooth0_traffic_bytes_per_launch"]


def cpu_baseline(p, gpu_iters: int, min_seconds: float = 10.0, flexible: bool = True):
    """The FP64 oracle, as it stands, on the host cores: whole solves of the
    same problem (1e-5 reduction from u0 = 0, the same beta as the GPU solve),
    repeated until at least min_seconds of CPU work have been timed."""
    from oracle import oracle as O
    g = O.Grid.from_problem(p)
    reps, dt, iters = 0, 0.0, 0
    while dt < min_seconds and reps < 20:
        t0 = time.perf_counter()
        u, st = O.pcg(g, p.f, rtol=p.rtol, flexible=flexible)
        dt += time.perf_counter() - t0
        reps += 1
        iters = st["iters"]
    return {"value": reps / dt, "unit": "solves/s", "cores": O.num_threads(), "kind": "oracle",
            "unknowns_iter_per_s": p.n * iters * reps / dt, "seconds": dt, "oracle_iters": iters,
            "sample": f"{reps} whole FP64 solves of the same {p.nx}x{p.ny}x{p.nz} problem "
                      f"(1e-5 reduction, {iters} iterations each, OpenMP over columns)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    if a.workload == "c2":
        return bench_c2(a)
    if a.workload == "robust":
        return bench_robust(a)
    if a.workload == "batch":
        return bench_batch(a)
    if a.workload == "serve":
        return bench_serve(a)
    import numpy as np
    import torch

    from paper_1307_2036_amd import ell, inputs, perfmodel

    torch.cuda.set_device(0)
    p = inputs.config1(n_levels=a.levels, nu_coarse=a.nu_coarse, nx=a.nx)
    schedule = ell.autotune(iters=4, **_desc_kw(p, a.precision)) if a.autotune else \
        ell.schedule_get(**_desc_kw(p, a.precision))
    G = ell.Grid.from_problem(p, precision=a.precision)
    f = torch.from_numpy(p.f).cuda()
    u = torch.zeros_like(f)
    n = p.n
    e = 8 if a.precision == "fp64" else 4
    # the plain FP64 solve uses the classic beta of Appendix B's PCG (the
    # V-cycle is symmetric); the mixed-precision preconditioner needs the
    # flexible one
    flexible = a.precision != "fp64"

    def step():
        u.zero_()
        return G.pcg_solve(f, u, rtol=p.rtol, maxiter=500, poll_every=8, flexible=flexible)

    if a.probe_copy:
        # a plain copy of known size: 2^25 doubles read and written once
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(a.warmup):
        _, st = step()
    torch.cuda.synchronize()
    _, st = step()
    iters = st.iters
    G.profile_enable(ell.ELL_K_SMOOTH0, 4 * (iters + 2) * a.steps + 64)
    G.profile_enable(ell.ELL_K_APPLY, (iters + 2) * a.steps + 16)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        _, st = step()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    assert st.status == 0, st

    def live(times):
        # launches enqueued after convergence return at once; keep the real ones
        med = float(np.median(times))
        return times[times > 0.25 * med]

    t_s = live(G.profile_times(ell.ELL_K_SMOOTH0))
    t_a = live(G.profile_times(ell.ELL_K_APPLY))
    feat = G.features
    dot_q = feat["fused_dots"] and flexible
    fpro = feat["fused_prolong"] and not flexible
    launch_bytes = (perfmodel.smooth0_launch_bytes(n, 8, fused_update=feat["fused_update"], dot_q=dot_q,
                                                   fused_prolong=fpro)
                    if a.precision == "fp64" else
                    perfmodel.smooth0_launch_bytes_hybrid(n, fused_update=feat["fused_update"], dot_q=dot_q))
    avg_ms = float(t_s.mean())
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    # the CG operator step reads z (and p_old after the first iteration) and writes
    # p_new, q: 24 B per unknown at K = 1, 32 B after; the steps of odd K >= 3 also
    # apply two deferred solution updates (u, p_old2 read, u written: 24 B more)
    apply_bytes = sum(24 if K == 1 else (56 if K % 2 else 32) for K in range(1, iters + 1)) / iters * n
    apply_gbs = apply_bytes / (float(t_a.mean()) * 1e-3) / 1e9
    cnt = int(t_s.size)

    solves = a.steps / elapsed
    it_bytes = perfmodel.pcg_iteration_bytes(n, G.levels, e, nu_coarse=p.nu_coarse, flexible=flexible,
                                             fused_update=feat["fused_update"], fused_dots=feat["fused_dots"],
                                             fused_prolong=fpro)
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": solves,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f64-outer/f32-vcycle",
        "data": "synthetic (seeded N(0,1) f, graded dz, log-normal lambda^2 profile)",
        "config": {"workload": f"gmg-pcg {p.nx}x{p.ny}x{p.nz} graded, omega2=1e-2, "
                               f"{G.levels} levels, nu_coarse={p.nu_coarse}, rtol 1e-5, u0=0",
                   "unknowns": n, "precision": a.precision, "parallelism": "single GPU",
                   "beta": "flexible" if flexible else "classic"},
        "iters": iters,
        "unknowns_iter_per_s": n * iters * solves,
        "hbm_gbs_algorithmic": it_bytes * iters * solves / 1e9,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "true_rel_residual": st.true_r_norm / st.b_norm,
        "roofline": {"bound": "hbm", "kernel": "finest-level line relaxation, " + (
                         ("k_smooth_seg_upd, k_smooth_tile_upd, k_smooth_tile_pro, k_smooth_tile_dot3, FP64"
                          if fpro else "k_smooth_seg(_upd), k_smooth_tile(_upd), k_smooth_tile_dot x2, FP64")
                         if a.precision == "fp64" else "FP32 pre / FP64 post sweeps") +
                     (" (residual update fused into the first pair)" if feat["fused_update"] else "") +
                     (" (finest prolongation fused into the first post sweep)" if fpro else ""),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(a.precision),
                     "avg_launch_us": avg_ms * 1e3, "launches": cnt,
                     "bytes_per_launch": launch_bytes},
        "cg_operator_kernel": {"kernel": "k_apply_dir_tile" if schedule["apply_tile"] else "k_apply_dir",
                               "achieved_gbs": apply_gbs, "avg_launch_us": float(t_a.mean()) * 1e3},
        "schedule": dict(schedule, autotuned=bool(a.autotune)),
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, iters, a.cpu_seconds, flexible)
    print(json.dumps(out), flush=True)


def _seq_fp64(problems, fs):
    """Plain FP64 single-grid solves one after another (the baseline)."""
    import torch
    from paper_1307_2036_amd import ell
    grids = [ell.Grid.from_problem(p) for p in problems]
    us = [torch.zeros_like(f) for f in fs]
    for g, f, u in zip(grids, fs, us):  # warm-up pass
        u.zero_()
        g.pcg_solve(f, u, rtol=1e-5, flexible=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for g, f, u in zip(grids, fs, us):
        u.zero_()
        _, st = g.pcg_solve(f, u, rtol=1e-5, flexible=False)
        iters.append(st.iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for g in grids:
        g.close()
    return len(problems) / dt, iters


def bench_batch(a):
    """64 uneven solves (nx in {64..256}, nz in {64, 96, 128}, log-uniform omega^2)
    advanced together by the batch engine with the FP32 preconditioner; one step
    = all 64 solves from u0 = 0 to 1e-5."""
    import numpy as np
    import torch
    from paper_1307_2036_amd import ell, inputs
    torch.cuda.set_device(0)
    ps = inputs.config3_instances(64)
    fs = [torch.from_numpy(p.f).cuda() for p in ps]
    n_total = sum(p.n for p in ps)
    prec = "fp32" if a.precision == "fp64" else a.precision
    ell.set_tuning(ell.ELL_TUNE_BATCH_GRAPH, a.batch_graph)
    B = ell.Batch(200 << 30)
    grids = [B.grid(p, precision=prec) for p in ps]
    us = [torch.zeros_like(f) for f in fs]

    def step():
        for u in us:
            u.zero_()
        return B.wait(B.submit(grids, fs, us, rtol=1e-5, poll_every=4))

    for _ in range(max(a.warmup, 1)):
        st = step()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        st = step()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(s.status == 0 for s in st)
    iters = [s.iters for s in st]
    solves = len(ps) * a.steps / elapsed
    seq, seq_iters = _seq_fp64(ps, fs)
    out = {
        "metric": METRIC, "value": solves, "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": elapsed / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64-outer/f32-vcycle",
        "data": "synthetic (64 seeded uneven instances)",
        "config": {"workload": "batch of 64 uneven gmg-pcg solves (nx in {64,96,128,192,256}, "
                               "nz in {64,96,128}, log-uniform omega2), grouped launches",
                   "unknowns_total": n_total, "precision": prec, "graph": a.batch_graph},
        "unknowns_iter_per_s": float(np.sum([p.n * it for p, it in zip(ps, iters)]) * a.steps / elapsed),
        "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
        "batch_ms_p50": float(np.percentile(np.array(lat) * 1e3, 50)),
        "fp64_sequential_solves_per_s": seq, "fp64_sequential_iters_mean": float(np.mean(seq_iters)),
        "speedup_vs_fp64_sequential": solves / seq,
    }
    print(json.dumps(out), flush=True)
    B.close()


def bench_c2(a):
    """Mixed precision at 1024x1024x128 (graded, standard depth), omega^2 swept
    over {1e-3, 1e-2, 1e-1}: per omega^2 the mixed-precision solve (BF16-rounded
    stencil coefficients, FP32 V-cycle, FP64 CG; or --precision fp32) and the
    plain FP64 solve to 1e-5, timed, plus the error of a tight (1e-12) mixed
    solve against the tight FP64 solve on the same GPU.  value = solves/s of the
    mixed path over the sweep (one solve per omega^2 per step)."""
    import numpy as np
    import torch
    from paper_1307_2036_amd import ell, inputs, perfmodel
    torch.cuda.set_device(0)
    prec = "bf16coef" if a.precision == "fp64" else a.precision
    rows, t_mixed, t_64 = [], 0.0, 0.0
    for omega2 in (1e-3, 1e-2, 1e-1):
        p = inputs.config2(omega2)
        f = torch.from_numpy(p.f).cuda()
        p.f = None
        u = torch.zeros_like(f)
        per = {}
        for name, pr in ((prec, prec), ("fp64", "fp64")):
            G = ell.Grid.from_problem(p, precision=pr)
            G.pcg_solve(f, u, rtol=p.rtol, flexible=pr != "fp64")  # warm-up
            times = []
            for _ in range(max(a.steps // 4, 2)):
                u.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = G.pcg_solve(f, u, rtol=p.rtol, poll_every=8, flexible=pr != "fp64")
                times.append(time.perf_counter() - t0)
            assert st.status == 0, st
            ut = torch.zeros_like(f)
            G.pcg_solve(f, ut, rtol=1e-12, maxiter=300)
            per[name] = dict(iters=st.iters, s=float(np.median(times)), tight=ut, levels=G.levels)
            G.close()
        e = 8 if prec == "fp64" else 4
        mixed_bytes = perfmodel.pcg_iteration_bytes(p.n, per[prec]["levels"], e) * per[prec]["iters"]
        err = float(torch.linalg.vector_norm(per[prec]["tight"] - per["fp64"]["tight"]) /
                    torch.linalg.vector_norm(per["fp64"]["tight"]))
        rows.append({"omega2": omega2, "levels": per[prec]["levels"], "iters_mixed": per[prec]["iters"],
                     "iters_fp64": per["fp64"]["iters"], "ms_mixed": per[prec]["s"] * 1e3,
                     "ms_fp64": per["fp64"]["s"] * 1e3,
                     "hbm_gbs_algorithmic_mixed": mixed_bytes / per[prec]["s"] / 1e9,
                     "tight_rel_err_vs_fp64": err})
        t_mixed += per[prec]["s"]
        t_64 += per["fp64"]["s"]
        del per, f, u
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": 3 / t_mixed, "unit": "solves/s", "n_gpus": 1, "steps": 3,
        "warmup": 1, "ms_per_step": t_mixed * 1e3 / 3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64-outer/f32-vcycle", "data": "synthetic (seeded N(0,1) f)",
        "config": {"workload": "gmg-pcg 1024x1024x128 graded, standard depth, omega2 in {1e-3,1e-2,1e-1}, "
                               "rtol 1e-5, u0=0", "unknowns": 1024 * 1024 * 128, "precision": prec},
        "fp64_solves_per_s": 3 / t_64, "speedup_vs_fp64": t_64 / t_mixed, "per_omega2": rows,
    }
    print(json.dumps(out), flush=True)


def bench_robust(a):
    """Robustness sweep of Sec. 7.3 (Table 7, 3.4e7 unknowns): the flat analogue
    of the paper's 512^2 x 128 run (Table 1 parameters: C_horiz = 17.8,
    lambda^2 = 0.0332, the paper's vertical grading with H = 1/100), omega^2
    scaled by f in {1, 10, 100} and lambda^2 by {1e-2, 1e2}; stand-alone
    multigrid with the standard depth (to one column), shallow (7 levels) and
    very shallow (4 levels, 5 coarsest-level sweeps) hierarchies, the one-level
    CG with block red/black SSOR line relaxation, and GMG-preconditioned CG
    (standard depth), each from u0 = 0 to 1e-5 in FP64.  value = solves/s of the
    standard stand-alone multigrid over the sweep."""
    import math
    import numpy as np
    import torch
    from paper_1307_2036_amd import ell, inputs
    torch.cuda.set_device(0)
    nx, nz = 512, 128
    h = math.pi / (2 * nx)
    dz = inputs.dz_paper_grading(nz, 0.01)
    f = torch.from_numpy(inputs.rhs_normal(nx, nx, dz, inputs.seed_for(1))).cuda()
    solvers = [("standard_mg", dict(n_levels=0, nu_coarse=1), "mg"),
               ("shallow_mg", dict(n_levels=7, nu_coarse=1), "mg"),
               ("very_shallow_mg", dict(n_levels=4, nu_coarse=5), "mg"),
               ("cg_line_relaxation", dict(n_levels=1, nu_coarse=0), "pcg"),
               ("gmg_pcg", dict(n_levels=0, nu_coarse=1), "pcg")]
    cases = [(1, 1), (1, 1e2), (1, 1e-2), (10, 1), (100, 1)]
    rows, t_std = [], 0.0
    for fw, fl in cases:
        row = {"f_omega2": fw, "f_lambda2": fl}
        for name, mg, kind in solvers:
            G = ell.Grid(nx, nx, nz, h, h, 17.8 * h * h * fw, dz,
                         np.full(nz, inputs.paper_lambda2(600.0) * fl), **mg)
            solve = G.mg_solve if kind == "mg" else G.pcg_solve
            u = torch.zeros_like(f)
            solve(f, u, rtol=1e-5, maxiter=1000)  # warm-up
            times = []
            for _ in range(2):
                u.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = solve(f, u, rtol=1e-5, maxiter=1000, poll_every=8)
                times.append(time.perf_counter() - t0)
            t = min(times)
            row[name] = {"iters": st.iters, "status": st.status, "levels": G.levels, "ms": t * 1e3,
                         "ms_per_iter": t * 1e3 / max(st.iters, 1)}
            if name == "standard_mg":
                t_std += t
            G.close()
        rows.append(row)
        print(json.dumps({"progress": row}), file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": len(cases) / t_std, "unit": "solves/s", "n_gpus": 1,
        "steps": len(cases), "warmup": 1, "ms_per_step": t_std * 1e3 / len(cases),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded N(0,1) f; the paper's Table 1 parameters on a flat periodic panel)",
        "config": {"workload": "robustness sweep 512x512x128 (Table 7): omega2 x {1,10,100}, "
                               "lambda2 x {1e-2,1e2}; standard/shallow/very shallow stand-alone GMG, "
                               "CG with line relaxation, GMG-PCG", "unknowns": nx * nx * nz},
        "paper_table7_iters": {"standard_mg": [6, 6, 6, 6, 8], "shallow_mg": [6, 6, 6, 6, 10],
                               "very_shallow_mg": [6, 6, 6, 15, 100],
                               "cg_line_relaxation": [43, 42, 42, 140, 300]},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def bench_serve(a):
    """Serving: Poisson arrivals of pressure solves on 24 resident streams
    (17 x 256^2, 6 x 512^2, 1 x 1024^2, nz = 128; uniform stream choice gives
    the 70/25/5 % mix), omega^2 in {1e-2, 5e-2}, fresh f ~ N(0,1) per request,
    warm start from the stream's previous solution, 1e-5 relative to ||b||,
    200 GB budget, FP32 preconditioner, continuous batching."""
    import numpy as np
    import torch
    from paper_1307_2036_amd import ell, inputs
    torch.cuda.set_device(0)
    rng = np.random.default_rng(inputs.seed_for(4))
    sizes = [256] * 17 + [512] * 6 + [1024]
    prec = "fp32" if a.precision == "fp64" else a.precision
    ell.set_tuning(ell.ELL_TUNE_BATCH_GRAPH, a.batch_graph)
    B = ell.Batch(200 << 30)
    streams = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(inputs.seed_for(4, stream=2))
    for idx, nx in enumerate(sizes):
        omega2 = float(rng.choice([1e-2, 5e-2]))
        p = inputs.graded_problem(f"stream{idx}", nx, 128, omega2, inputs.seed_for(4, idx),
                                  inputs.seed_for(4, idx, stream=1), with_f=False)
        g = B.grid(p, precision=prec)
        shape = (p.nz, p.ny, p.nx)
        w = torch.from_numpy(p.dz).cuda().view(-1, 1, 1)
        streams.append(dict(p=p, g=g, u=torch.zeros(shape, dtype=torch.float64, device="cuda"),
                            f=torch.empty(shape, dtype=torch.float64, device="cuda"), w=w))

    def new_rhs(s):
        # in place: the stream's previous request has finished when this runs
        # (four passes over f: the draw, the per-level sums, the subtraction)
        f = s["f"]
        torch.randn(f.shape, generator=gen, device="cuda", dtype=torch.float64, out=f)
        f -= (f.sum(dim=(1, 2)) * s["w"].view(-1)).sum() / (s["w"].sum() * f.shape[1] * f.shape[2])

    def run(duration, rate):
        """rate None: closed loop (every stream always has one request)."""
        pending = {}
        done_lat, done_iters = [], []
        t_start = time.perf_counter()
        next_arrival = t_start
        queue_per_stream = [[] for _ in streams]  # arrivals waiting for their stream
        busy = [False] * len(streams)
        n_done = 0
        while True:
            now = time.perf_counter()
            if now - t_start > duration:
                break
            if rate is None:
                for i, s in enumerate(streams):
                    if not busy[i]:
                        queue_per_stream[i].append(now)
            else:
                while next_arrival <= now:
                    i = int(rng.integers(len(streams)))
                    queue_per_stream[i].append(next_arrival)
                    next_arrival += rng.exponential(1.0 / rate)
            for i, s in enumerate(streams):
                if not busy[i] and queue_per_stream[i]:
                    t_arr = queue_per_stream[i].pop(0)
                    new_rhs(s)
                    t = B.submit([s["g"]], [s["f"]], [s["u"]], rtol=1e-5, rel_to_rhs=True, poll_every=1)
                    pending[t] = (i, t_arr)
                    busy[i] = True
            for t in list(pending):
                r = B.poll(t)
                if r is not None:
                    i, t_arr = pending.pop(t)
                    B.wait(t)
                    done_lat.append(time.perf_counter() - t_arr)
                    done_iters.append(r[0].iters)
                    busy[i] = False
                    n_done += 1
            time.sleep(0.0002)
        for t in list(pending):
            B.wait(t)
        elapsed = time.perf_counter() - t_start
        return n_done / elapsed, np.array(done_lat) * 1e3, done_iters

    run(2.0, None)  # warm-up: every stream solved at least once
    capacity, _, _ = run(a.serve_seconds / 2, None)
    rate = a.serve_load * capacity
    thr, lat, iters = run(a.serve_seconds, rate)
    # plain FP64 sequential baseline on the same GPU: for each size class, a few
    # requests with the same semantics (fresh f generated on the GPU as in the
    # serving loop, warm start, 1e-5 of ||b||) solved one after another with the
    # single-grid FP64 path; mix-weighted
    classes = {256: 17 / 24, 512: 6 / 24, 1024: 1 / 24}
    t_class = {}
    for nx, wgt in classes.items():
        s0 = next(s for s in streams if s["p"].nx == nx)
        G = ell.Grid.from_problem(s0["p"])
        u = torch.zeros_like(s0["u"])
        new_rhs(s0)
        G.pcg_solve(s0["f"], u, rtol=1e-5, rel_to_rhs=True, flexible=False)
        torch.cuda.synchronize()
        times = []
        for _ in range(9):  # the median of nine warm-started requests per size
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            new_rhs(s0)
            G.pcg_solve(s0["f"], u, rtol=1e-5, rel_to_rhs=True, flexible=False)
            times.append(time.perf_counter() - t0)
        t_class[nx] = float(np.median(times))
        G.close()
    seq = 1.0 / sum(w * t_class[nx] for nx, w in classes.items())
    out = {
        "metric": METRIC, "value": thr, "unit": "solves/s", "n_gpus": 1, "steps": len(lat),
        "warmup": 0, "ms_per_step": 1e3 / thr if thr else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64-outer/f32-vcycle",
        "data": "synthetic (seeded Poisson arrivals, fresh N(0,1) f per request)",
        "config": {"workload": "serving: 24 streams (17x256^2, 6x512^2, 1x1024^2, nz=128), "
                               "Poisson arrivals, warm starts, continuous batching, 200 GB budget",
                   "arrival_rate_per_s": rate, "load": a.serve_load, "precision": prec,
                   "graph": a.batch_graph},
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "closed_loop_capacity_solves_per_s": capacity,
        "iters_mean": float(np.mean(iters)) if iters else None,
        "hbm_resident_gb": B.bytes_in_use() / 1e9,
        "fp64_sequential_solves_per_s": seq,
        "fp64_sequential_ms_by_size": {str(k): v * 1e3 for k, v in t_class.items()},
        "speedup_vs_fp64_sequential": thr / seq,
        "capacity_speedup_vs_fp64_sequential": capacity / seq,
    }
    print(json.dumps(out), flush=True)
    B.close()


if __name__ == "__main__":
    main()
