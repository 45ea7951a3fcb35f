"""Serving harness: drive a Server with a timed arrival stream.

Arrivals are replayed on the host's wall clock: before each step every query
whose arrival time has passed is submitted (while slots are free), then one
step runs; a query's latency is the wall time from its arrival to the end of
the step that finished it.

Command line (the seeded serving stream; two phases so that each fits one
run of a few minutes):

    python -m paper_1008_3171_amd.serving burst  --count 20000 --out burst.json
    python -m paper_1008_3171_amd.serving stream --count 20000 --burst burst.json --record rec.json

`burst` submits every query at once and reports capacity (queries/s) and the
results; `stream` replays the same queries as Poisson arrivals at rho times
that capacity, reports p50/p99 latency and checks every result against the
burst's. `--record` also writes the stream's summary, a SHA-256 over all its
results, and the results of every query with n <= 10^5 plus a seeded sample
of 300 with 10^5 < n <= 10^7, small enough to check against an independent
CPU evaluation.
"""
from __future__ import annotations

import argparse
import collections
import json
import sys
import time


def run_stream(server, stream, time_scale: float = 1.0, progress=None):
    """stream: [(t_arrival, formula, n, nbits, P)] sorted by t_arrival.
    progress(done, total, seconds) is called after steps that finish queries,
    at most every 10 s. Returns (results {tag: (S, code, nterms)},
    latencies [s], makespan [s], steps)."""
    pending = collections.deque(enumerate(stream))
    arrival = {}
    results = {}
    lat = []
    steps = 0
    t0 = time.perf_counter()
    last = t0
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
        if progress is not None and time.perf_counter() - last >= 10.0:
            last = time.perf_counter()
            progress(len(results), len(stream), last - t0)
    makespan = time.perf_counter() - t0
    return results, lat, makespan, steps


def results_digest(queries, results) -> str:
    """SHA-256 over every (tag, formula, n, nbits, P, S, code, N), in tag order."""
    import hashlib
    h = hashlib.sha256()
    for tag in sorted(results):
        ta, f, n, w, P = queries[tag]
        S, code, N = results[tag]
        h.update(("%d %d %d %d %d %x %d %d\n" % (tag, f, n, w, P, S, code, N)).encode())
    return h.hexdigest()


def write_record(path, summary, queries, results, burst):
    import random
    small = [t for t in sorted(results) if queries[t][2] <= 10 ** 5]
    mid = [t for t in sorted(results) if 10 ** 5 < queries[t][2] <= 10 ** 7]
    pick = sorted(small + random.Random(3171).sample(mid, min(300, len(mid))))
    rec = dict(summary)
    rec["burst"] = {k: burst[k] for k in ("makespan_s", "capacity_qps", "terms_per_s", "steps")}
    rec["results_sha256"] = results_digest(queries, results)
    rec["checked_results"] = [[t, queries[t][1], queries[t][2], queries[t][3], queries[t][4],
                               "%x" % results[t][0], results[t][1], results[t][2]] for t in pick]
    with open(path, "w") as f:
        json.dump(rec, f, indent=0)


def percentile(xs, p):
    if not xs:
        return float("nan")
    s = sorted(xs)
    i = min(len(s) - 1, max(0, int(round(p / 100.0 * (len(s) - 1)))))
    return s[i]


def _log(done, total, t):
    print("%d/%d queries done, %.0f s" % (done, total, t), file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1008_3171_amd.serving")
    ap.add_argument("phase", choices=["burst", "stream"])
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=3171)
    ap.add_argument("--lo-exp", type=float, default=3.0)
    ap.add_argument("--hi-exp", type=float, default=11.0)
    ap.add_argument("--rho", type=float, default=0.8)
    ap.add_argument("--out", help="burst: where to write capacity and results")
    ap.add_argument("--burst", help="stream: the burst phase's output file")
    ap.add_argument("--step-terms", type=int, default=1 << 30)
    ap.add_argument("--record", help="stream: where to write the summary and checkable results")
    args = ap.parse_args(argv)

    import paper_1008_3171_amd as pb
    from paper_1008_3171_amd import workloads
    base = workloads.serving_stream(args.count, seed=args.seed, lo_exp=args.lo_exp,
                                    hi_exp=args.hi_exp, rate=1.0)
    terms = sum(pb.head_terms(f, n) for _, f, n, _, _ in base)
    srv = pb.Server(max_active=1024, step_terms=args.step_terms)
    rec = {"queries": args.count, "head_terms": terms, "seed": args.seed,
           "workload": "n = floor(10^U), U ~ U(%g, %g), BBP/Bellard 1/2 each, w in {64, 256}, "
                       "P = w + 64, numpy PCG64 seed %d" % (args.lo_exp, args.hi_exp, args.seed)}
    if args.phase == "burst":
        res, lat, mk, steps = run_stream(srv, [(0.0,) + q[1:] for q in base], progress=_log)
        rec.update({"phase": "burst", "makespan_s": mk, "capacity_qps": args.count / mk,
                    "terms_per_s": terms / mk, "steps": steps,
                    "all_certified": all(v[1] == pb.PI_OK for v in res.values()),
                    "results": {str(t): ["%x" % S, code, N] for t, (S, code, N) in res.items()}})
        if args.out:
            with open(args.out, "w") as f:
                json.dump(rec, f)
        rec.pop("results")
    else:
        with open(args.burst) as f:
            burst = json.load(f)
        lam = args.rho * burst["capacity_qps"]
        res, lat, mk, steps = run_stream(srv, base, time_scale=1.0 / lam, progress=_log)
        same = all(burst["results"][str(t)] == ["%x" % S, code, N] for t, (S, code, N) in res.items())
        rec.update({"phase": "stream", "capacity_qps": burst["capacity_qps"], "rho": args.rho,
                    "rate_qps": lam, "makespan_s": mk, "qps": args.count / mk,
                    "terms_per_s": terms / mk, "steps": steps,
                    "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
                    "identical_to_burst": same and len(res) == len(burst["results"]),
                    "all_certified": all(v[1] == pb.PI_OK for v in res.values())})
        if args.record:
            write_record(args.record, rec, base, res, burst)
    srv.close()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
