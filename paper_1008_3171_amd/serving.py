"""Serving harness: drive a Server with a timed arrival stream.

Arrivals are replayed on the host's wall clock: before each step every query
whose arrival time has passed is submitted (while slots are free), then one
step runs; a query's latency is the wall time from its arrival to the end of
the step that finished it.
"""
from __future__ import annotations

import collections
import time


def run_stream(server, stream, time_scale: float = 1.0):
    """stream: [(t_arrival, formula, n, nbits, P)] sorted by t_arrival.
    Returns (results {tag: (S, code, nterms)}, latencies [s], makespan [s], steps)."""
    pending = collections.deque(enumerate(stream))
    arrival = {}
    results = {}
    lat = []
    steps = 0
    t0 = time.perf_counter()
    while pending or server.active():
        now = time.perf_counter() - t0
        while pending and pending[0][1][0] * time_scale <= now:
            tag, (ta, f, n, w, P) = pending[0]
            if not server.submit(f, n, w, P, tag):
                break
            arrival[tag] = ta * time_scale
            pending.popleft()
        if server.active() == 0:
            if pending:
                wait = pending[0][1][0] * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            continue
        server.step()
        steps += 1
        done_at = time.perf_counter() - t0
        for tag, S, code, N in server.poll():
            results[tag] = (S, code, N)
            lat.append(done_at - arrival[tag])
    makespan = time.perf_counter() - t0
    return results, lat, makespan, steps


def percentile(xs, p):
    if not xs:
        return float("nan")
    s = sorted(xs)
    i = min(len(s) - 1, max(0, int(round(p / 100.0 * (len(s) - 1)))))
    return s[i]
