"""Host logic of the serving loop (paper_1307_2036_amd/serve.py) on the CPU:
per-stream FIFO order, one request in flight per stream, arrival-to-result
latency, closed-loop throughput, draining, and the Poisson arrival process.
A fake engine stands in for the GPU: each solve completes a fixed virtual
time after its submission."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1307_2036_amd import serve as S


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self, dt=1e-3):
        self.t += dt


class FakeEngine:
    """Completes a solve `work[stream]` virtual seconds after its submission;
    checks that a stream never has two solves in flight."""

    def __init__(self, clock, work):
        self.clock, self.work = clock, work
        self.next = 0
        self.live = {}
        self.log = []     # (event, stream, time)

    def submit(self, i):
        assert all(s != i for s, _ in self.live.values()), "two requests of one stream in flight"
        t = self.next
        self.next += 1
        self.live[t] = (i, self.clock())
        self.log.append(("submit", i, self.clock()))
        return t

    def poll(self, t):
        i, ts = self.live[t]
        if self.clock() + 1e-12 >= ts + self.work[i]:
            return SimpleNamespace(iters=3 + i, status=0)
        return None

    def release(self, t):
        i, _ = self.live.pop(t)
        self.log.append(("release", i, self.clock()))


def loop(work, n=None):
    clk = Clock()
    eng = FakeEngine(clk, work)
    return S.ServingLoop(n or len(work), eng, clock=clk, idle=clk.tick), eng, clk


def test_fifo_latency_bookkeeping():
    """Three requests of one stream arriving at 0, 1 and 2 ms with a 5 ms
    solve: each is submitted when the previous one has been released, and the
    latencies are 5, 10 and 15 ms (arrival to result)."""
    L, eng, clk = loop({0: 5e-3})
    arr = S.ScriptedArrivals([(0.0, 0), (1e-3, 0), (2e-3, 0)])
    done, elapsed, backlog = L.run(1.0, arr, until_served=3)
    assert backlog == 0 and [r.stream for r in done] == [0, 0, 0]
    assert [round(r.t_arrival * 1e3, 6) for r in done] == [0.0, 1.0, 2.0]
    assert [round(r.latency * 1e3, 6) for r in done] == [5.0, 10.0, 15.0]
    assert all(r.iters == 3 and r.status == 0 for r in done)
    # each submission follows the release of the stream's previous request
    subs = [t for e, _, t in eng.log if e == "submit"]
    rels = [t for e, _, t in eng.log if e == "release"]
    assert all(s >= r for s, r in zip(subs[1:], rels[:-1]))


def test_streams_overlap_and_late_admission():
    """A request on another stream that arrives while a long solve runs is
    submitted at once (it does not wait for the running solve)."""
    L, eng, clk = loop({0: 20e-3, 1: 3e-3})
    arr = S.ScriptedArrivals([(0.0, 0), (4e-3, 1), (5e-3, 0)])
    done, _, _ = L.run(1.0, arr, until_served=3)
    by = {(r.stream, round(r.t_arrival * 1e3, 6)): r for r in done}
    late = by[(1, 4.0)]
    assert round(late.t_submit * 1e3, 6) == 4.0 and round(late.latency * 1e3, 6) == 3.0
    assert round(by[(0, 0.0)].latency * 1e3, 6) == 20.0
    # the second request of stream 0 waited for the first (FIFO, warm start)
    second = by[(0, 5.0)]
    assert second.t_submit >= by[(0, 0.0)].t_done
    assert [r.stream for r in done] == [1, 0, 0]


def test_closed_loop_throughput_and_drain():
    """Closed loop: every idle stream gets a request at once.  Two streams of
    4 and 6 ms solves, each occupied for one more 1 ms loop turn per request,
    serve about 1/5 + 1/7 requests per ms; requests still in flight at the end
    are drained and counted as backlog, not as served."""
    L, eng, clk = loop({0: 4e-3, 1: 6e-3})
    done, elapsed, backlog = L.run(0.2, None)
    # a solve occupies its stream from its submission to the poll that sees
    # it finished, plus one loop turn (1 ms) before the next submission
    expect = elapsed * (1 / 5e-3 + 1 / 7e-3)
    assert abs(len(done) - expect) <= 3, (len(done), expect)
    assert backlog <= 2
    assert not eng.live, "in-flight tickets were not drained"
    s = S.summary(done, elapsed)
    assert s["served"] == len(done) and s["failed"] == 0
    assert math.isclose(s["solves_per_s"], len(done) / elapsed)
    lat = sorted(r.latency for r in done)
    assert s["p50_ms"] == pytest.approx(np.percentile(np.array(lat) * 1e3, 50))
    assert 4.0 <= s["p50_ms"] <= 6.0 + 1e-9


def test_poisson_arrivals():
    rng = np.random.default_rng(123)
    arr = S.PoissonArrivals(500.0, 4, rng, t0=10.0)
    got = arr.due(10.0 + 20.0)
    ts = np.array([t for t, _ in got])
    assert np.all(np.diff(ts) >= 0) and ts[0] >= 10.0 and ts[-1] <= 30.0
    # 10000 expected arrivals: the count and the mean gap are within 4 sigma
    assert abs(len(got) - 10000) <= 4 * math.sqrt(10000)
    assert abs(np.diff(ts).mean() - 1 / 500.0) <= 4 * (1 / 500.0) / math.sqrt(len(ts))
    streams = np.bincount([i for _, i in got], minlength=4)
    assert streams.min() > 0.9 * len(got) / 4
    assert arr.due(30.0) == []  # nothing is returned twice
    with pytest.raises(ValueError):
        S.PoissonArrivals(0.0, 2, rng)


def test_poisson_served_latency_includes_queueing():
    """Arrivals faster than one stream can serve: the queue grows and the
    latency of the k-th request grows with k."""
    L, eng, clk = loop({0: 10e-3})
    arr = S.ScriptedArrivals([(k * 2e-3, 0) for k in range(10)])
    done, _, backlog = L.run(1.0, arr, until_served=10)
    lat = [r.latency for r in done]
    assert all(b > a for a, b in zip(lat, lat[1:]))
    assert backlog == 0
