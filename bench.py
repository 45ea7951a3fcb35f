#!/usr/bin/env python3
"""Benchmark: modexp terms/s of one bit-extraction query on one MI355X.

A step is one whole pi_extract_ex call: Bellard's formula (eq (1.2)) at bit
position n = 10^12 with 256 result bits and P = 320 (five 64-bit limbs),
about 7.0e11 head terms with moduli below 2^40, plus the tail, the
reduction and the certification. Inputs are the query parameters
themselves; nothing is read from disk.

Prints one JSON line. `value` = head terms per second of the timed steps.
`roofline` prices the head kernel's data-path instructions against the
chip's VALU issue rate, next to the counter-derived figures of the committed
profile and the int32-multiply fraction of the algorithmic multiply count;
`cpu_baseline` is the oracle on a bounded seeded sub-slice of the same
workload, on every host core this process may use.

The arithmetic: exact binary64 (integer-valued doubles, every operation
proven exact) for moduli from 2^29 to 2^51 plus 32- and 64-bit integers,
hence `dtype` "binary64-exact+u32/u64"; `integer_only` repeats the query with
integer Montgomery arithmetic for every modulus (dtype "u32/u64").
"""
from __future__ import annotations

import argparse
import json
import os
import random
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz: the VALU issue rate.
# v_fma_f64 (78.6 TFLOP/s = this rate x 2 flops) and v_mad_u64_u32 both issue
# at it on gfx950, so the head kernel is priced in VALU lane-operations.
PEAK_VALU = 256 * 64 * 2.4e9

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "head_kernel_bellard_n1e12_P320_traffic.json")
# SQ_INSTS_VALU of the headline head kernel, per arithmetic mode, from
# rocprofv3 --pmc runs of this script (profiles/head_kernel_*_counters.md)
COUNTERS_FILE = os.path.join(ROOT, "profiles", "head_kernel_bellard_n1e12_P320_counters.json")
# the head kernel's device code and the planner that sizes its chunks (the
# chunk count sets the scheduler's atomics, hence the write traffic)
KERNEL_SOURCES = ["kernels.hip", "arith.h", "plan.h", "abi.cpp", "host.h"]


def kernel_source_hash():
    """sha256 over the sources of the head kernel and its launch planning."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1008_3171_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the headline head kernel, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs recorded in profiles/, each scaled by the
    factor a plain 1 GiB copy gives the same counter; None when the kernel
    sources changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t["fetch_kib"] * 1024 * t["fetch_factor"] + t["write_kib"] * 1024 * t["write_factor"]


def measured_counters(arith):
    """VALU wave instructions per launch of the headline head kernel in one
    arithmetic mode ("fast" or "integer"), from the committed counter runs;
    None when the kernel sources changed after they were taken."""
    try:
        with open(COUNTERS_FILE) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return c.get(arith)


def series(formula):
    # (c, a, b) per series and the step; the sign does not change the work
    if formula == 1:
        return [(2, 10, 1), (0, 10, 3), (-4, 10, 5), (-4, 10, 7), (-6, 10, 9), (-1, 4, 1),
                (-6, 4, 3)], 10
    return [(2, 8, 1), (-1, 2, 1), (0, 8, 5), (-1, 4, 3)], 4


def _pre_bits(run, Mmin, Mmax, a):
    """Exponent bits the library folds into a class-62 segment's start value
    (the planner's rule: the start value g 2^v must satisfy (g 2^v)^2 < 2^60 M
    and g 2^v < 2^56, with g < (2^63 a run / M^2 + 2) M)."""
    for pre in (3, 2, 1):
        shift = 2.0 ** ((1 << pre) - 1)
        good = True
        for M in (float(Mmin), float(Mmax)):
            g = (a * run * 2.0 ** 63 / (M * M) + 2.0) * M * shift
            if g * g >= M * 2.0 ** 60 or g >= 2.0 ** 56:
                good = False
        if good:
            return pre
    return 0


# VALU instructions of the head kernel's data path per head term, from the
# compiled gfx950 code (loop control and scheduling excluded). A term's ladder
# runs over the bits of its exponent X, minus the bits its start value takes
# (binary64: the top 6; class 62: `pre`; class 32: none). X is E for the
# binary64 classes and E + 64L + offset for the integer ones, whose Hensel
# division needs 2^(64L) r. Each of the remaining r bits costs one squaring,
# each whole W-bit window its digit (2 instructions when folded into the last
# squaring, 5 when applied after it) and a short leading window (r mod W
# bits) one more than a whole one, for its 64-bit shift. The per-term part covers the start value, the
# reciprocal or the 32-bit inverse and the division at L = 5 (binary64: long
# division; integer: Hensel, mask and accumulation).
#   (name, first modulus, W, per squaring, per window, per term, offset)
# (binary64 per term at L = 5: seven 46-bit digits of 5 instructions each.)
KERNEL_CLASSES = [
    ("22", 0, 3, 3, 2, 70, -32),        # R = 2^32 Montgomery, doubling start
    ("27", 2 ** 22, 2, 3, 2, 62, -32),  # R = 2^32, run-quotient start
    ("29", 2 ** 27, 1, 3, 2, 62, -32),  # R = 2^32, run-quotient start
    ("f4", 2 ** 29, 4, 6, 2, 49, 0),    # binary64
    ("f3", 2 ** 33, 3, 6, 2, 48, 0),
    ("f2", 2 ** 42, 2, 6, 2, 47, 0),
    ("fs", 2 ** 48, 5, 6, 5, 47, 0),    # binary64, digit applied after the squarings
    ("62", 2 ** 51, 1, 16, 0, 104, -62),  # R = 2^62, two 31-bit digits
]
# The binary64 classes also take a carry step over each lane's digit sums
# every 120 terms (28 instructions at L = 5) and add the sums to the lane's
# limbs once per run of 256 (81).
FP_EXTRA_PER_TERM = 28 / 120 + 81 / 256


def _term_ops(cls, W, per_sq, per_win, fixed, nb, pre):
    start = 6 if cls[0] == "f" else (pre if cls == "62" else 0)
    r = max(0, nb - start)
    flush = FP_EXTRA_PER_TERM if cls[0] == "f" else 0.0
    return fixed + flush + per_sq * r + per_win * (r // W) + (per_win + 1 if r % W else 0)


def valu_ops_per_launch(formula, n, P, run=64):
    """Data-path VALU instructions of every head term of one extraction (the
    per-term model above, summed over the bands of equal bitlen(X) of each
    series and modulus class). Returns (ops, head terms)."""
    rows, step = series(formula)
    L = (P + 63) // 64
    d = n - 1
    total = 0
    terms = 0
    for c, a, b in rows:
        if d + c < 0:
            continue
        K = (d + c) // step + 1

        def first_k(mlim):
            return min(K, max(0, -(-(mlim - b) // a)))

        bounds = [first_k(m) for _, m, _, _, _, _, _ in KERNEL_CLASSES] + [K]
        for i, (cls, _, W, per_sq, per_win, fixed, off) in enumerate(KERNEL_CLASSES):
            lo, hi = bounds[i], bounds[i + 1]
            if lo >= hi:
                continue
            pre = 0
            if cls == "62":
                pre = _pre_bits(min(run, max(1, (hi - lo) // 1024)), a * lo + b,
                                a * (hi - 1) + b, a)
            base = d + c + (0 if cls[0] == "f" else 64 * L + off)
            k = lo
            while k < hi:
                X = base - step * k
                bl = X.bit_length()
                lowX = 1 << (bl - 1) if bl > 0 else 0
                kmax = min(hi - 1, (base - lowX) // step) if bl > 0 else hi - 1
                cnt = kmax - k + 1
                total += cnt * _term_ops(cls, W, per_sq, per_win, fixed, bl, pre)
                terms += cnt
                k = kmax + 1
    return int(round(total)), terms


def mul32_per_launch(formula, n, P):
    """The algorithmic 32-bit multiply count of every head term of one
    extraction, as the work unit of the int32-multiply roofline: a term with
    exponent E is bitlen(E) - 1 modular squarings of a 64-bit residue at 10
    32-bit multiplies each (four partial products and six for the reduction),
    16 for -M^-1 mod 2^64, and 7 per limb of the L-limb division, less 4
    saved at the ends. Returns (multiplies, head terms)."""
    rows, step = series(formula)
    L = (P + 63) // 64
    d = n - 1
    total = terms = 0
    for c, a, b in rows:
        if d + c < 0:
            continue
        K = (d + c) // step + 1
        k = 0
        while k < K:
            E = d + c - step * k
            bl = E.bit_length()
            lowE = 1 << (bl - 1) if bl > 0 else 0
            kmax = min(K - 1, (d + c - lowE) // step) if bl > 0 else K - 1
            cnt = kmax - k + 1
            total += cnt * (10 * max(bl - 1, 0) + 16 + 7 * L - 4)
            terms += cnt
            k = kmax + 1
    return total, terms


def host_cores():
    """(threads to use, what the host shows): the CPUs this process may run
    on, further capped by a cgroup CPU quota when one is set, with nproc and
    the CPU model."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()
        if q != "max":
            quota = max(1, int(int(q) / int(per)))
    except (OSError, ValueError):
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = min(usable, quota) if quota else usable
    return threads, {"nproc": os.cpu_count(), "affinity": usable, "cgroup_quota_cpus": quota,
                     "cpu_model": model}


def cpu_baseline(formula, n, P, target_s=12.0):
    """The oracle on a seeded sub-slice: equal-length random k ranges of every
    series, sized from a short probe to take about target_s seconds."""
    import oracle
    threads, host = host_cores()
    rows, step = series(formula)
    rng = random.Random(1008)
    d = n - 1

    def run(length):
        t0 = time.perf_counter()
        done = 0
        for j, (c, a, b) in enumerate(rows):
            K = (d + c) // step + 1
            k0 = rng.randrange(0, max(1, K - length))
            oracle.sum_slice(formula, j, d, k0, k0 + length, P, threads)
            done += length
        return done, time.perf_counter() - t0

    done, dt = run(1 << 16)
    per_term = dt / done
    length = int(max(1 << 16, min(1 << 26, target_s / per_term / len(rows))))
    done, dt = run(length)
    return {"value": done / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
            "per_core": done / dt / threads, "host": host,
            "sample": "%d series x %d consecutive k at seeded random offsets of the same "
                      "query (%d head terms, %.1f s)" % (len(rows), length, done, dt)}


def batch_vs_loop(pb, torch, count=4096, seed=1008):
    """The seeded 4096-query batch as one pi_extract_batch call and as
    a loop of pi_extract_ex calls (one query per launch) on the same stream.
    Both are timed with HIP events on that stream; outputs must be identical."""
    from paper_1008_3171_amd import workloads
    specs = workloads.batch_queries(count, seed=seed)
    stream = torch.cuda.current_stream()
    qarr, total = pb.make_queries(specs)
    out_b = torch.zeros(total, dtype=torch.int64, device="cuda")
    st_b = torch.zeros(4 * count, dtype=torch.int32, device="cuda")
    out_l = torch.zeros(total, dtype=torch.int64, device="cuda")
    st_l = torch.zeros(4 * count, dtype=torch.int32, device="cuda")
    nbytes = pb.workspace_size(qarr, count)
    ws = torch.zeros((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
    terms = sum(pb.head_terms(f, n) for f, n, _, _ in specs)

    def batch():
        pb.extract_batch(qarr, count, out_b, st_b, workspace=ws, stream=stream)

    def loop():
        for i, (f, n, w, P) in enumerate(specs):
            off = qarr[i].out_offset
            L = pb.limbs(P)
            pb.extract(f, n, w, P, out=out_l[off:off + L], status=st_l[4 * i:4 * i + 4],
                       stream=stream)

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3, time.perf_counter() - t0

    batch(); loop(); torch.cuda.synchronize()        # warm up both paths
    tb, wb = timed(batch)
    tl, wl = timed(loop)
    same = bool(torch.equal(out_b, out_l) and torch.equal(st_b, st_l))
    # the same batch as a plan captured once into a HIP graph, then replayed
    out_g = torch.zeros(total, dtype=torch.int64, device="cuda")
    st_g = torch.zeros(4 * count, dtype=torch.int32, device="cuda")
    plan = pb.BatchPlan(qarr, count, out_g, st_g)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        plan.launch(stream=side)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch(stream=torch.cuda.current_stream())
    graph.replay()
    tg, wg = timed(graph.replay)
    same_graph = bool(torch.equal(out_b, out_g) and torch.equal(st_b, st_g))
    plan.close()
    certified = all(pb.status_of(st_b, i)[0] == pb.PI_OK for i in range(count))
    print("batch vs loop done", file=sys.stderr, flush=True)
    return {"queries": count, "head_terms": terms, "batch_s": tb, "loop_s": tl,
            "batch_queries_per_s": count / tb, "loop_queries_per_s": count / tl,
            "speedup": tl / tb, "batch_terms_per_s": terms / tb,
            "graph_replay_s": tg, "graph_speedup": tl / tg, "graph_identical": same_graph,
            "batch_wall_s": wb, "loop_wall_s": wl, "identical_outputs": same,
            "all_certified": certified,
            "workload": "Bellard, n = floor(10^U), U ~ U(4, 9), w in {32,64,128,256}, "
                        "P = w + 64, numpy PCG64 seed %d" % seed}


def serving_bench(pb, torch, count=1000, seed=3171, hi_exp=10.0, rho=0.8):
    """The serving stream, scaled: `count` queries of the seeded serving stream
    (n = floor(10^U), U ~ U(3, hi_exp), BBP or Bellard 50/50, w in {64, 256},
    P = w + 64). First every query arrives at once, which measures capacity
    (queries/s); then the same queries arrive as a Poisson stream at rho times
    that capacity, and latency = completion - arrival is recorded."""
    from paper_1008_3171_amd import serving, workloads
    base = workloads.serving_stream(count, seed=seed, hi_exp=hi_exp, rate=1.0)
    burst = [(0.0,) + q[1:] for q in base]
    srv = pb.Server(max_active=1024, step_terms=1 << 30)
    res0, lat0, mk0, st0 = serving.run_stream(srv, burst)
    capacity = count / mk0
    lam = rho * capacity
    res1, lat1, mk1, st1 = serving.run_stream(srv, base, time_scale=1.0 / lam)
    # the same stream with unpipelined steps (each step waited for before
    # the next is planned): lower latency, the device idles while planning
    srv.set_pipeline(0)
    res2, lat2, mk2, st2 = serving.run_stream(srv, base, time_scale=1.0 / lam)
    srv.close()
    terms = sum(pb.head_terms(f, n) for _, f, n, _, _ in base)
    print("serving done", file=sys.stderr, flush=True)
    return {"queries": count, "head_terms": terms, "capacity_qps": capacity,
            "burst_makespan_s": mk0, "rate_qps": lam, "rho": rho,
            "makespan_s": mk1, "qps": count / mk1, "terms_per_s": terms / mk1,
            "p50_latency_s": serving.percentile(lat1, 50),
            "p99_latency_s": serving.percentile(lat1, 99),
            "steps": st1, "identical_to_burst": res0 == res1 and res0 == res2,
            "unpipelined": {"qps": count / mk2, "p50_latency_s": serving.percentile(lat2, 50),
                            "p99_latency_s": serving.percentile(lat2, 99), "steps": st2},
            "all_certified": all(v[1] == pb.PI_OK for v in res1.values()),
            "workload": "n = floor(10^U), U ~ U(3, %g), BBP/Bellard 1/2 each, w in {64, 256}, "
                        "P = w + 64, numpy PCG64 seed %d, Poisson arrivals" % (hi_exp, seed),
            "scaled": "a %d-query stream of the same recipe with n up to 10^%g, so that the "
                      "benchmark stays within minutes; the full stream (20,000 queries, n up to "
                      "10^11, about 25 GPU-minutes) runs as python -m "
                      "paper_1008_3171_amd.serving burst|stream" % (count, hi_exp)}


def paper_slice(pb, torch):
    """The paper-scale slice: Bellard at n = 2*10^15, k in [10^14, 10^14 + 2^32)
    for all seven series (moduli near 2^50), as seven pi_sum_slice calls."""
    stream = torch.cuda.current_stream()
    n, P = 2 * 10 ** 15, 320
    k0, k1 = 10 ** 14, 10 ** 14 + 2 ** 32
    outs = [torch.zeros(pb.limbs(P), dtype=torch.int64, device="cuda") for _ in range(7)]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for rep in range(2):                       # the first pass warms up
        torch.cuda.synchronize()
        e0.record(stream)
        for j in range(7):
            pb.sum_slice(pb.term_id(pb.BELLARD, j), n, k0, k1, P, out=outs[j], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    return {"n": n, "k0": k0, "k1": k1, "terms": 7 * (k1 - k0), "seconds": s,
            "terms_per_s": 7 * (k1 - k0) / s}


def integer_only(pb, torch, formula, n, w, P, fast_ms):
    """The headline query again with pi_set_arith(PI_ARITH_INTEGER): integer
    Montgomery arithmetic for every modulus, same bits."""
    stream = torch.cuda.current_stream()
    out = torch.zeros(pb.limbs(P), dtype=torch.int64, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    pb.set_arith(pb.ARITH_INTEGER)
    try:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        pb.extract(formula, n, w, P, out=out, status=st, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
    finally:
        pb.set_arith(pb.ARITH_FAST)
    ms = e0.elapsed_time(e1)
    terms = pb.head_terms(formula, n)
    headline = (formula, n, w, P) == (pb.BELLARD, 10 ** 12, 256, 320)
    rf = {"bound": "alu", "peak": PEAK_VALU / 1e12, "unit": "T VALU lane-ops/s"}
    rf.update(multiply_and_counter_fractions("integer", formula, n, P, terms, ms * 1e-3,
                                             headline))
    rf["achieved"] = rf.get("counter_lane_ops_per_s")
    rf["frac"] = rf.get("issue_frac_counters")
    return {"ms": ms, "terms_per_s": terms / (ms * 1e-3), "fast_over_integer": ms / fast_ms,
            "dtype": "u32/u64", "roofline": rf,
            "S": "%x" % pb.to_int(out, P), "certified": pb.status_of(st)[0] == pb.PI_OK}


def multiply_and_counter_fractions(arith, formula, n, P, terms, seconds, headline):
    """The int32-multiply roofline of the algorithmic multiply count (a
    multiply-add per lane per clock: full rate on gfx950, by the probe in
    profiles/valu_rates.md), and, for the headline query, VALU instructions
    per term and the issue fraction from the committed SQ_INSTS_VALU count."""
    mul, mterms = mul32_per_launch(formula, n, P)
    assert mterms == terms
    out = {"mul32_per_term": mul / terms, "mul32_frac": mul / seconds / PEAK_VALU,
           "valu_per_term_counters": None, "issue_frac_counters": None,
           "counter_lane_ops_per_s": None}
    c = measured_counters(arith) if headline else None
    if c:
        lane_ops = c["sq_insts_valu"] * 64.0
        out["valu_per_term_counters"] = lane_ops / terms
        out["counter_lane_ops_per_s"] = lane_ops / seconds / 1e12
        out["issue_frac_counters"] = lane_ops / seconds / PEAK_VALU
    return out


def other_workloads(pb, torch):
    """Smaller single queries: Bellard n = 10^6 (64 bits, P = 96),
    Bellard and BBP at n = 10^10 (256 bits, P = 320)."""
    stream = torch.cuda.current_stream()
    rows = {}
    for name, f, n, w, P in (("bellard_n1e6_P96", pb.BELLARD, 10 ** 6, 64, 96),
                             ("bellard_n1e10_P320", pb.BELLARD, 10 ** 10, 256, 320),
                             ("bbp_n1e10_P320", pb.BBP, 10 ** 10, 256, 320)):
        out = torch.zeros(pb.limbs(P), dtype=torch.int64, device="cuda")
        st = torch.zeros(4, dtype=torch.int32, device="cuda")
        pb.extract(f, n, w, P, out=out, status=st, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        pb.extract(f, n, w, P, out=out, status=st, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        terms = pb.head_terms(f, n)
        S = pb.to_int(out, P)
        rows[name] = {"seconds": sec, "head_terms": terms, "terms_per_s": terms / sec,
                      "certified": pb.status_of(st)[0] == pb.PI_OK,
                      "hex": "%0*x" % ((w + 3) // 4, S >> (P - w))}
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=10 ** 12)
    ap.add_argument("--nbits", type=int, default=256)
    ap.add_argument("--P", type=int, default=320)
    ap.add_argument("--formula", choices=["bellard", "bbp"], default="bellard")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-integer", action="store_true",
                    help="skip timing the query again in integer-only arithmetic")
    ap.add_argument("--arith", choices=["fast", "integer"], default="fast",
                    help="arithmetic of the timed steps: exact binary64 where cheaper (the "
                         "default) or integer Montgomery for every modulus")
    ap.add_argument("--measure-peak", action="store_true",
                    help="run the VALU issue-rate probe and report its rates")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device twice (a plain copy "
                         "kernel of known size, to calibrate memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path has no multi-GPU code (a query's index "
              "ranges would shard across GPUs with one exchange of its carry-save counters, "
              "80 bytes at P = 320, at the end); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1008_3171_amd as pb

    formula = pb.BELLARD if args.formula == "bellard" else pb.BBP
    n, w, P = args.n, args.nbits, args.P
    stream = torch.cuda.current_stream()
    if args.arith == "integer":
        pb.set_arith(pb.ARITH_INTEGER)
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 17, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = torch.zeros(pb.limbs(P), dtype=torch.int64, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        pb.extract(formula, n, w, P, out=out, status=st, stream=stream)
        torch.cuda.synchronize()
        print("warmup step done", file=sys.stderr, flush=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        pb.extract(formula, n, w, P, out=out, status=st, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    code, N = pb.status_of(st)
    S = pb.to_int(out, P)
    print("timed steps done", file=sys.stderr, flush=True)

    ops, terms = valu_ops_per_launch(formula, n, P)
    assert terms == pb.head_terms(formula, n)
    headline = (formula, n, w, P) == (pb.BELLARD, 10 ** 12, 256, 320)
    value = terms / (ms * 1e-3)
    achieved = ops / (ms * 1e-3)
    rec = {
        "metric": "modexp terms/s at n=1e12, 256-bit exact",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64" if args.arith == "integer" else "binary64-exact+u32/u64",
        "data": "synthetic",
        "config": {"workload": "single query, %s formula, n=%d, %d result bits, P=%d"
                               % (args.formula, n, w, P),
                   "head_terms": terms, "limbs": pb.limbs(P)},
        "certified": code == pb.PI_OK,
        "nterms": N,
        "result_hex": "%0*x" % ((w + 3) // 4, S >> (P - w)),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12,
                     "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_VALU,
                     "traffic": measured_traffic() if headline and args.arith == "fast" else None,
                     "valu_ops_per_launch": ops, "valu_per_term_model": ops / terms},
    }
    rec["roofline"].update(multiply_and_counter_fractions(args.arith, formula, n, P, terms,
                                                          ms * 1e-3, headline))
    if args.arith == "integer":
        # the per-term instruction model describes the default arithmetic only
        for key in ("achieved", "frac", "valu_ops_per_launch", "valu_per_term_model"):
            rec["roofline"][key] = None
        rec["roofline"]["achieved"] = rec["roofline"]["counter_lane_ops_per_s"]
        rec["roofline"]["frac"] = rec["roofline"]["issue_frac_counters"]
        rec["arith"] = "integer"
    if n == 10 ** 12 and w == 256 and formula == pb.BELLARD:
        # Table 2.2, m = 12 starts at 10^12 + 1: our bits 1..255
        import re
        row = open(os.path.join(ROOT, "tests", "golden", "table_2_2.txt")).read()
        h = re.search(r"^12 \d+ \d+ ([0-9A-F]+)$", row, re.M).group(1)
        ref = int(h, 16) >> (4 * len(h) - 255)
        rec["matches_table_2_2_m12"] = ((S >> (P - w)) & ((1 << 255) - 1)) == ref
    if not args.no_integer and args.arith == "fast":
        io = integer_only(pb, torch, formula, n, w, P, ms)
        io["same_bits"] = io.pop("S") == "%x" % S
        rec["integer_only"] = io
    if args.measure_peak:
        import subprocess
        probe = os.path.join(ROOT, "paper_1008_3171_amd", "probe", "valu_rates")
        res = subprocess.run([probe], capture_output=True, text=True, timeout=120, check=True)
        rec["valu_rates"] = [json.loads(l) for l in res.stdout.splitlines() if l.strip()]
    if not args.no_batch:
        rec["other_workloads"] = other_workloads(pb, torch)
        rec["batch"] = batch_vs_loop(pb, torch)
        rec["paper_slice"] = paper_slice(pb, torch)
    if not args.no_serving:
        rec["serving"] = serving_bench(pb, torch)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(formula, n, P)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
