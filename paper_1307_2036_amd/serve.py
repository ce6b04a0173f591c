"""Serving loop for pressure-correction solves (beyond the paper).

Requests arrive on a fixed set of streams (a stream is one resident grid with
its multigrid hierarchy and its last solution, as a forecast model keeps one
pressure problem per domain).  Each stream serves its requests first in, first
out; a request warm-starts from the stream's previous solution.  The loop
submits a stream's next request as soon as the stream is idle, so requests
that arrive while others are on the GPU join the batch engine's running
iterations at its next cycle (continuous batching: the engine advances every
active solve with one grouped launch per stage and retires each as it
converges).  Latency is measured from a request's arrival to the moment its
result is known on the host.

The loop itself holds no GPU code: it drives an engine object with three
calls, so its queueing and bookkeeping run (and are tested) on the CPU.

  engine.submit(stream) -> ticket   build the request's right-hand side and
                                    submit the solve, warm start from the
                                    stream's current solution
  engine.poll(ticket) -> result     None while the solve runs, else an object
                                    with .iters and .status
  engine.release(ticket)            the ticket's result has been consumed

``BatchEngine`` is the engine over ``ell.Batch`` used by the benchmark.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Request:
    stream: int
    t_arrival: float
    t_submit: float = math.nan
    t_done: float = math.nan
    iters: int = -1
    status: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class PoissonArrivals:
    """Arrival times of a Poisson process of the given rate (per second),
    starting at t0, each request on a stream drawn uniformly from n_streams."""

    def __init__(self, rate: float, n_streams: int, rng: np.random.Generator, t0: float = 0.0):
        if not rate > 0:
            raise ValueError("rate must be > 0")
        self.rate = rate
        self.n = n_streams
        self.rng = rng
        self.next_t = t0 + rng.exponential(1.0 / rate)

    def due(self, now: float):
        """Arrivals with time <= now, in time order: a list of (t, stream)."""
        out = []
        while self.next_t <= now:
            out.append((self.next_t, int(self.rng.integers(self.n))))
            self.next_t += self.rng.exponential(1.0 / self.rate)
        return out


class ScriptedArrivals:
    """Arrivals at fixed offsets (seconds) from the first call of due(), each
    on a given stream: a deterministic trace, e.g. for tests."""

    def __init__(self, events):
        self.events = sorted((float(t), int(i)) for t, i in events)
        self.k = 0
        self.t0 = None

    def due(self, now: float):
        if self.t0 is None:
            self.t0 = now
        out = []
        while self.k < len(self.events) and self.t0 + self.events[self.k][0] <= now:
            t, i = self.events[self.k]
            out.append((self.t0 + t, i))
            self.k += 1
        return out


class ServingLoop:
    """Per-stream FIFO queues over an engine (see the module docstring).

    run(duration, arrivals, until_served): arrivals None is the closed loop
    (every idle stream has a request waiting, the capacity measurement);
    otherwise an object with due(now) -> [(t_arrival, stream)].  The run ends
    after duration seconds, or once until_served requests have been served.
    Requests still running at the end are waited for but not counted as
    served within the window; returns (served requests in completion order,
    elapsed seconds, requests left queued or in flight at the end)."""

    def __init__(self, n_streams: int, engine, clock: Callable[[], float] = time.perf_counter,
                 idle: Optional[Callable[[], None]] = None):
        self.n = n_streams
        self.engine = engine
        self.clock = clock
        self.idle = idle if idle is not None else (lambda: time.sleep(2e-4))

    def run(self, duration: float, arrivals=None, until_served: Optional[int] = None):
        queues = [deque() for _ in range(self.n)]
        in_flight = {}           # ticket -> Request
        busy = [False] * self.n
        done: List[Request] = []
        t0 = self.clock()
        while True:
            now = self.clock()
            if now - t0 > duration or (until_served is not None and len(done) >= until_served):
                break
            if arrivals is None:
                for i in range(self.n):
                    if not busy[i] and not queues[i]:
                        queues[i].append(Request(i, now))
            else:
                for t, i in arrivals.due(now):
                    queues[i].append(Request(i, t))
            for i in range(self.n):
                if not busy[i] and queues[i]:
                    req = queues[i].popleft()
                    req.t_submit = self.clock()
                    in_flight[self.engine.submit(i)] = req
                    busy[i] = True
            for t in list(in_flight):
                res = self.engine.poll(t)
                if res is not None:
                    req = in_flight.pop(t)
                    req.t_done = self.clock()
                    req.iters, req.status = int(res.iters), int(res.status)
                    self.engine.release(t)
                    busy[req.stream] = False
                    done.append(req)
            self.idle()
        elapsed = self.clock() - t0
        for t in list(in_flight):   # drain: the engine must not be left with work
            while self.engine.poll(t) is None:
                self.idle()
            self.engine.release(t)
        backlog = sum(len(q) for q in queues) + len(in_flight)
        return done, elapsed, backlog


def summary(done: List[Request], elapsed: float) -> dict:
    """Throughput and arrival-to-result latency of the requests served."""
    lat = np.array([r.latency for r in done]) * 1e3
    return {"served": len(done), "seconds": elapsed,
            "solves_per_s": len(done) / elapsed if elapsed > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "iters_mean": float(np.mean([r.iters for r in done])) if done else None,
            "failed": sum(1 for r in done if r.status != 0)}


class BatchEngine:
    """Engine over ``ell.Batch``: one resident grid per stream, the stream's
    solution kept on the device for the next warm start, and each request's
    right-hand side f ~ N(0, 1) with its volume-weighted mean removed drawn on
    the device (in place: the stream's previous request has finished when the
    next one is submitted).  Solves stop at rtol relative to ||b|| (the warm
    start makes ||r_0|| meaningless as a reference).

    on_submit(stream, f, u) / on_done(stream, u, stats), if given, see the
    request's device vectors before it is submitted and after it finished
    (the tests copy them out to check every served result)."""

    def __init__(self, batch, problems, precision="fp32", rtol=1e-5, maxiter=500, seed=0,
                 flexible=True, poll_every=1, on_submit=None, on_done=None):
        import torch
        self.torch = torch
        self.B = batch
        self.rtol, self.maxiter, self.flexible, self.poll_every = rtol, maxiter, flexible, poll_every
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)
        self.streams = []
        for p in problems:
            g = batch.grid(p, precision=precision)
            shape = (p.nz, p.ny, p.nx)
            w = torch.from_numpy(np.asarray(p.dz, dtype=np.float64)).cuda()
            self.streams.append(dict(p=p, g=g, w=w,
                                     u=torch.zeros(shape, dtype=torch.float64, device="cuda"),
                                     f=torch.empty(shape, dtype=torch.float64, device="cuda")))
        self.on_submit, self.on_done = on_submit, on_done
        self.owner = {}

    def new_rhs(self, s):
        f, w = s["f"], s["w"]
        self.torch.randn(f.shape, generator=self.gen, device="cuda", dtype=self.torch.float64, out=f)
        f -= (f.sum(dim=(1, 2)) * w).sum() / (w.sum() * f.shape[1] * f.shape[2])

    def submit(self, i: int) -> int:
        s = self.streams[i]
        self.new_rhs(s)
        if self.on_submit:
            self.on_submit(i, s["f"], s["u"])
        t = self.B.submit([s["g"]], [s["f"]], [s["u"]], rtol=self.rtol, maxiter=self.maxiter,
                          flexible=self.flexible, rel_to_rhs=True, poll_every=self.poll_every)
        self.owner[t] = i
        return t

    def poll(self, t: int):
        r = self.B.poll(t)
        return None if r is None else r[0]

    def release(self, t: int):
        st = self.B.wait(t, check=False)[0]
        i = self.owner.pop(t)
        if self.on_done:
            self.on_done(i, self.streams[i]["u"], st)

    def close(self):
        for s in self.streams:
            s["g"].close()
        self.streams = []
