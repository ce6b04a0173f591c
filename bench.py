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
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain device copy of a 268 MB vector (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum seconds of oracle work in the CPU-baseline sample")
    return ap.parse_args()


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


def cpu_baseline(p, gpu_iters: int, min_seconds: float = 10.0):
    """The FP64 oracle, as it stands, on the host cores: whole solves of the
    same problem (1e-5 reduction from u0 = 0), repeated until at least
    min_seconds of CPU work have been timed."""
    from oracle import oracle as O
    g = O.Grid.from_problem(p)
    reps, dt, iters = 0, 0.0, 0
    while dt < min_seconds and reps < 20:
        t0 = time.perf_counter()
        u, st = O.pcg(g, p.f, rtol=p.rtol)
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
    import numpy as np
    import torch

    from paper_1307_2036_amd import ell, inputs, perfmodel

    torch.cuda.set_device(0)
    p = inputs.config1(n_levels=a.levels, nu_coarse=a.nu_coarse, nx=a.nx)
    G = ell.Grid.from_problem(p, precision=a.precision)
    f = torch.from_numpy(p.f).cuda()
    u = torch.zeros_like(f)
    n = p.n
    e = 8 if a.precision == "fp64" else 4

    def step():
        u.zero_()
        return G.pcg_solve(f, u, rtol=p.rtol, maxiter=500, poll_every=8)

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
    launch_bytes = (perfmodel.smooth0_launch_bytes(n, 8) if a.precision == "fp64"
                    else perfmodel.smooth0_launch_bytes_hybrid(n))
    avg_ms = float(t_s.mean())
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    # the CG operator step reads z, p_old, u and writes p_new, q, u (48 B per unknown)
    apply_gbs = 48 * n / (float(t_a.mean()) * 1e-3) / 1e9
    cnt = int(t_s.size)

    solves = a.steps / elapsed
    it_bytes = perfmodel.pcg_iteration_bytes(n, G.levels, e, nu_coarse=p.nu_coarse)
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
                   "unknowns": n, "precision": a.precision, "parallelism": "single GPU"},
        "iters": iters,
        "unknowns_iter_per_s": n * iters * solves,
        "hbm_gbs_algorithmic": it_bytes * iters * solves / 1e9,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "true_rel_residual": st.true_r_norm / st.b_norm,
        "roofline": {"bound": "hbm", "kernel": f"k_smooth_seg (finest level, {'FP64' if a.precision == 'fp64' else 'FP32 pre / FP64 post'})",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(a.precision),
                     "avg_launch_us": avg_ms * 1e3, "launches": cnt,
                     "bytes_per_launch": launch_bytes},
        "cg_operator_kernel": {"kernel": "k_apply_dir", "achieved_gbs": apply_gbs,
                               "avg_launch_us": float(t_a.mean()) * 1e3},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, iters, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
