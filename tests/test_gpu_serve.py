"""The serving loop on the GPU (paper_1307_2036_amd/serve.py over the batch
engine): a short trace with a request admitted while others run and requests
that warm-start from their stream's previous result.  Every served result is
checked against the FP64 oracle started from the same initial guess with the
same right-hand side: at the same iteration count to 1e-10 for FP64 serving,
solved tightly (rtol 1e-12) to 1e-8 for the FP32 preconditioner, and at the
production tolerance within two iterations of the oracle and 1e-4 of its
solution."""
import numpy as np
import pytest
import torch

from paper_1307_2036_amd import inputs as I
from paper_1307_2036_amd import serve as S
from solve_parity import check_solve

pytestmark = pytest.mark.gpu


def problems():
    # stream 0 is the largest, so the others are admitted while it runs
    return [I.graded_problem("s0", 128, 48, 1e-2, 51, 52),
            I.graded_problem("s1", 64, 32, 5e-2, 53, 54),
            I.graded_problem("s2", 32, 24, 1e-2, 55, 56, n_levels=3, nu_coarse=5)]


# two requests on stream 0 (the second warm-starts), stream 1 arriving while
# stream 0 runs, stream 2 later, then second requests on streams 1 and 2
TRACE = [(0.0, 0), (0.0, 0), (0.002, 1), (0.004, 2), (0.006, 1), (0.008, 2)]


def serve_trace(E, precision, rtol):
    subs, outs = [], []
    B = E.Batch(8 << 30)
    eng = S.BatchEngine(B, problems(), precision=precision, rtol=rtol, maxiter=400, seed=7,
                        flexible=True, poll_every=1,
                        on_submit=lambda i, f, u: subs.append((i, f.cpu().numpy(), u.cpu().numpy())),
                        on_done=lambda i, u, st: outs.append((i, u.cpu().numpy(), st)))
    loop = S.ServingLoop(len(eng.streams), eng)
    done, elapsed, backlog = loop.run(120.0, S.ScriptedArrivals(TRACE), until_served=len(TRACE))
    eng.close()
    B.close()
    assert backlog == 0 and len(done) == len(TRACE) == len(subs) == len(outs)
    # pair each submission with its result (per stream, in order)
    per = {}
    for i, f, u0 in subs:
        per.setdefault(i, []).append([f, u0])
    k = {}
    pairs = []
    for i, u, st in outs:
        j = k.get(i, 0)
        k[i] = j + 1
        f, u0 = per[i][j]
        pairs.append((i, j, f, u0, u, st))
    return done, pairs


@pytest.fixture(scope="module")
def E():
    from paper_1307_2036_amd import ell
    return ell


def test_served_fp64_results_match_oracle(E, orc):
    done, pairs = serve_trace(E, "fp64", 1e-5)
    ps = problems()
    warm = 0
    for i, j, f, u0, u, st in pairs:
        assert st.status == 0, (i, j, st)
        if j > 0:
            warm += 1
            assert np.abs(u0).max() > 0  # warm start from the stream's previous solution
        g = orc.Grid.from_problem(ps[i])
        info = check_solve(orc, g, f, u, st, 1e-5, u0=u0, rel_to_rhs=True, flexible=True)
        print("stream", i, "request", j, info)
    assert warm == 3


def test_served_fp32_validation_mode_matches_oracle(E, orc):
    """FP32 preconditioner, validation mode: served to rtol 1e-12 of ||b||,
    each result within 1e-8 of the oracle's tight solve from the same start."""
    done, pairs = serve_trace(E, "fp32", 1e-12)
    ps = problems()
    for i, j, f, u0, u, st in pairs:
        assert st.status == 0, (i, j, st)
        g = orc.Grid.from_problem(ps[i])
        u_ref, st_ref = orc.pcg(g, f, u0=u0, rtol=1e-12, maxiter=400, rel_to_rhs=True)
        err = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
        print("stream", i, "request", j, "iters", st.iters, st_ref["iters"], "rel", err)
        assert err <= 1e-8, (i, j, err)


def test_served_fp32_production_tolerance(E, orc):
    done, pairs = serve_trace(E, "fp32", 1e-5)
    ps = problems()
    for i, j, f, u0, u, st in pairs:
        assert st.status == 0
        g = orc.Grid.from_problem(ps[i])
        u_ref, st_ref = orc.pcg(g, f, u0=u0, rtol=1e-5, rel_to_rhs=True)
        assert st.iters <= st_ref["iters"] + 2, (i, j, st.iters, st_ref["iters"])
        assert np.linalg.norm(u - u_ref) <= 1e-4 * np.linalg.norm(u_ref), (i, j)
    s = S.summary(done, 1.0)
    assert s["served"] == len(TRACE) and s["failed"] == 0
