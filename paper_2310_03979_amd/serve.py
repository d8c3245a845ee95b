"""Arrival replay: replays an arrival schedule against a ``Server`` and
reports per-request latency and throughput.

Arrivals are given as offsets in seconds; a request is submitted when the
wall clock passes its arrival time, the server is stepped continuously, and a
request's latency runs from its arrival time to the moment the replay loop sees
its completion (polled, ~0.2 ms resolution).
"""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (requests/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def replay(server, requests: Sequence[dict], arrivals: Sequence[float], timeout_s: float = 600.0,
           progress=None, progress_every_s: float = 10.0) -> dict:
    """requests: dicts with plan, seed, out, b2_scale, spectrum (see Server.submit).
    ``progress(msg)`` is called about every ``progress_every_s`` seconds."""
    n = len(requests)
    order = np.argsort(np.asarray(arrivals), kind="stable")
    tickets = {}
    done_at = {}
    t0 = time.perf_counter()
    last = 0.0
    nxt = 0
    while len(done_at) < n:
        now = time.perf_counter() - t0
        if progress is not None and now - last >= progress_every_s:
            last = now
            progress(f"t={now:.1f}s submitted {nxt}/{n} completed {len(done_at)}/{n}")
        if now > timeout_s:
            raise TimeoutError(f"serving replay exceeded {timeout_s} s ({len(done_at)}/{n} done)")
        while nxt < n and arrivals[order[nxt]] <= now:
            i = int(order[nxt])
            r = requests[i]
            tickets[server.submit(r["plan"], r["seed"], r["out"], r.get("b2_scale", 1.0),
                                  spectrum=r.get("spectrum"))] = i
            nxt += 1
        st = server.step()
        got = server.poll()
        tnow = time.perf_counter() - t0
        for t in got:
            done_at[tickets[t]] = tnow
        if not got and not st["launched"]:
            time.sleep(0.0002)
    makespan = max(done_at.values()) - float(min(arrivals))
    lat = np.array([done_at[i] - arrivals[i] for i in range(n)])
    return dict(latency=lat, makespan=makespan, p50=float(np.percentile(lat, 50)),
                p99=float(np.percentile(lat, 99)), mean=float(lat.mean()))
