"""Open-loop request driver for the continuous-batching server.

Requests arrive as a Poisson process: inter-arrival gaps are exponential with
mean 1/rate, drawn from a seeded generator.  The loop submits each request
once its arrival time has passed and otherwise keeps ticking the server, so
new requests join while earlier ones are still iterating on the device.  All
scheduling, sigma launches and Davidson steps happen inside the library; this
loop only moves arrivals into it and reads the results back.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import CANCELLED, DONE, FAILED, Server


@dataclass
class Served:
    rid: int
    arrival: float          # scheduled arrival, seconds after the start
    latency: float          # completion - submission (seconds)
    wait: float             # admission - submission (seconds)
    state: int
    energies: np.ndarray
    resid: np.ndarray
    n_iter: int
    n_dets: int
    sigma_vectors: int
    extra: dict = field(default_factory=dict)


def arrival_times(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process with the given rate."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=n)
    return np.cumsum(gaps) - gaps[0]


def run(server: Server, requests, arrivals=None, idle_sleep: float = 1e-4):
    """Serve `requests` (dicts of Server.submit keyword arguments) arriving at
    `arrivals` (seconds; None: all at once).  Returns (list of Served in
    request order, wall seconds from the first arrival to the last
    completion)."""
    n = len(requests)
    arrivals = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=float)
    order = np.argsort(arrivals, kind="stable")
    rids = [None] * n
    nxt = 0
    pending = 0
    t0 = time.monotonic()
    while nxt < n or pending > 0:
        now = time.monotonic() - t0
        while nxt < n and arrivals[order[nxt]] <= now:
            j = int(order[nxt])
            rids[j] = server.submit(**requests[j])
            nxt += 1
            pending += 1
        if pending > 0:
            left, _ = server.tick()
            pending = left
        elif nxt < n:
            time.sleep(min(idle_sleep, max(0.0, arrivals[order[nxt]] - (time.monotonic() - t0))))
    wall = time.monotonic() - t0
    out = []
    for j in range(n):
        r = server.result(rids[j])
        nd, _, _, sv = server.request_info(rids[j])
        out.append(Served(rids[j], float(arrivals[j]), r.t_done - r.t_submit, r.t_admit - r.t_submit, r.state,
                          r.energies, r.resid, r.n_iter, nd, sv))
    return out, wall


def summary(served, wall: float) -> dict:
    """p50/p99 latency, throughput and counts of a finished run."""
    lat = np.array([s.latency for s in served if s.state == DONE])
    return dict(
        requests=len(served),
        done=int(sum(s.state == DONE for s in served)),
        failed=int(sum(s.state == FAILED for s in served)),
        cancelled=int(sum(s.state == CANCELLED for s in served)),
        p50_s=float(np.percentile(lat, 50)) if lat.size else None,
        p99_s=float(np.percentile(lat, 99)) if lat.size else None,
        wall_s=wall,
        requests_per_s=len(lat) / wall if wall > 0 else None,
    )
