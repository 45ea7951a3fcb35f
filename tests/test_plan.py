"""The host planner, through pi_plan_head (CPU only: nothing is launched).

A query's head indices are split per series into segments by modulus range,
each with the arithmetic its moduli allow, and into chunks of 256 * run
indices. For many queries and slices, in both arithmetic modes:
- each series' segments tile exactly the head part of the requested range;
- every modulus of a segment lies in the range its class is built for;
- the chunk counts agree with the runs, and a query stays below 2^31 chunks;
- the Montgomery start values the kernels form from one quotient per lane run
  stay inside their bounds, checked in exact integers for sampled lanes:
  2^32 - qM < 2M (run-quotient classes) and, for R = 2^62,
  (g 2^v)^2 < 2^60 M and g 2^v < 2^56 with g = 2^62 - qM and v < 2^pre.
"""
import ctypes
import random

import pytest

import oracle
import paper_1008_3171_amd as pb

# modulus range [2^lo, 2^hi) per class, in the order the planner cuts them
FAST = [(22, 0, 22), (27, 22, 27), (29, 27, 29), (33, 29, 33), (42, 33, 42), (48, 42, 48),
        (51, 48, 51), (64, 51, 54)]
INTEGER = [(22, 0, 22), (27, 22, 27), (29, 27, 29), (31, 29, 31), (64, 31, 36), (64, 36, 54)]


def head_range(formula, j, n, k0, k1):
    rows, step, _ = oracle.series_table(formula)
    s, c, a, b = rows[j]
    K = (n - 1 + c) // step + 1 if n - 1 + c >= 0 else 0
    return max(0, k0), min(k1, K), a, b


def lane_moduli(rng, a, b, kb, ke, run):
    # first moduli of sampled lane runs: both ends of the segment and random
    ks = {kb, min(ke - 1, kb + 1), ke - 1, max(kb, ke - 1 - 2 * (run - 1))}
    ks |= {rng.randrange(kb, ke) for _ in range(6)}
    return [a * k + b for k in sorted(ks)]


def check_plan(formula, mask, n, k0, k1, P, table, rng):
    segs = pb.plan_head(formula, n, P, k0, k1, mask)
    rows, step, _ = oracle.series_table(formula)
    total_chunks = 0
    for j in range(len(rows)):
        mine = [g for g in segs if g["j"] == j]
        lo, hi, a, b = head_range(formula, j, n, k0, k1)
        if not (mask >> j) & 1 or lo >= hi:
            assert mine == [], (formula, j, n, k0, k1)
            continue
        # the segments tile [lo, hi) in order
        assert mine[0]["kb"] == lo and mine[-1]["ke"] == hi
        for g, h in zip(mine, mine[1:]):
            assert g["ke"] == h["kb"]
        for g in mine:
            kb, ke, run, cls = g["kb"], g["ke"], g["run"], g["cls"]
            assert kb < ke and run >= 1
            Mmin, Mmax = a * kb + b, a * (ke - 1) + b
            ranges = [(lo2, hi2) for c, lo2, hi2 in table if c == cls]
            assert ranges, cls
            assert any(Mmin >= (1 << lo2 if lo2 else 0) and Mmax < 1 << hi2
                       for lo2, hi2 in ranges), (cls, Mmin, Mmax)
            assert g["nchunks"] == -(-(ke - kb) // (256 * run))
            total_chunks += g["nchunks"]
            dM = 2 * a
            if cls in (27, 29, 31):
                for M in lane_moduli(rng, a, b, kb, ke, run):
                    q = (1 << 32) // (M + dM * (run - 1))
                    assert 0 <= (1 << 32) - q * M < 2 * M, (cls, M, run)
            if cls == 64:
                v = (1 << g["pre"]) - 1
                for M in lane_moduli(rng, a, b, kb, ke, run):
                    q = (1 << 62) // (M + dM * (run - 1))
                    assert q < 1 << 32
                    gs = ((1 << 62) - q * M) << v
                    assert gs * gs < M << 60 and gs < 1 << 56, (M, run, g["pre"])
            else:
                assert g["pre"] == 0
    assert total_chunks < 1 << 31
    return segs


def queries(rng):
    out = []
    for f in (pb.BBP, pb.BELLARD):
        for n in (1, 2, 9, 1000, 10 ** 6, 10 ** 9 + 7, 10 ** 10, 10 ** 12, 2 * 10 ** 15):
            out.append((f, 0x7F, n, 0, 2 ** 64 - 1, rng.choice([1, 64, 96, 320, 1088])))
        rows, step, _ = oracle.series_table(f)
        for _ in range(60):
            j = rng.randrange(len(rows))
            s, c, a, b = rows[j]
            e = rng.uniform(3, 53.9)
            kc = int(2 ** e) // a
            n = min(2 ** 61, step * (kc + rng.randrange(0, 10 ** 7)) + rng.randrange(1, 10 ** 6))
            k0 = max(0, kc - rng.randrange(0, 10 ** 6))
            k1 = min((2 ** 54 - 1 - b) // a + 1, k0 + rng.randrange(0, 10 ** 9))
            out.append((f, 1 << j, n, k0, k1, rng.randrange(1, 1089)))
    return out


@pytest.mark.parametrize("mode,table", [(pb.ARITH_FAST, FAST), (pb.ARITH_INTEGER, INTEGER)])
def test_plans_tile_the_head_and_respect_every_class_bound(mode, table):
    rng = random.Random(8 + mode)
    pb.set_arith(mode)
    try:
        for q in queries(rng):
            check_plan(*q, table, rng)
    finally:
        pb.set_arith(pb.ARITH_FAST)


def test_headline_plan():
    # n = 10^12: every Bellard series reaches the three-bit binary64 class
    # (moduli up to 10^12 < 2^40) and no modulus reaches 2^42
    segs = check_plan(pb.BELLARD, 0x7F, 10 ** 12, 0, 2 ** 64 - 1, 320, FAST, random.Random(1))
    assert {g["cls"] for g in segs} == {22, 27, 29, 33, 42}
    assert sum(g["ke"] - g["kb"] for g in segs) == pb.head_terms(pb.BELLARD, 10 ** 12)


def test_long_runs_for_huge_slices():
    # 2^53 indices of BBP's 2k+1 series must stay below 2^31 chunks: runs grow
    # past the largest run cap the tuning accepts
    rows, step, _ = oracle.series_table(pb.BBP)
    s, c, a, b = rows[1]
    k1 = (2 ** 54 - 1 - b) // a + 1
    k0 = k1 - 2 ** 53
    segs = check_plan(pb.BBP, 2, 2 ** 61, k0, k1, 64, FAST, random.Random(2))
    assert max(g["run"] for g in segs) > 4096


def test_plan_errors():
    lib = pb.load()
    count = ctypes.c_int(-7)
    # too small an output array: the count is still reported
    assert lib.pi_plan_head(pb.BELLARD, 0x7F, 10 ** 6, 0, 2 ** 64 - 1, 96, None, 0,
                            ctypes.byref(count)) == pb.PI_EINVAL
    assert count.value == len(pb.plan_head(pb.BELLARD, 10 ** 6, 96)) > 0
    count.value = -7
    assert lib.pi_plan_head(5, 1, 10 ** 6, 0, 10, 96, None, 0, ctypes.byref(count)) == pb.PI_EINVAL
    assert lib.pi_plan_head(pb.BBP, 1, 0, 0, 10, 96, None, 0, ctypes.byref(count)) == pb.PI_EINVAL
    assert lib.pi_plan_head(pb.BBP, 1, 10, 0, 10, 0, None, 0, ctypes.byref(count)) == pb.PI_EINVAL
    assert lib.pi_plan_head(pb.BBP, 1, 10, 0, 10, 96, None, 0, None) == pb.PI_EINVAL
    assert count.value == -7
    # moduli past 2^54 are refused
    assert lib.pi_plan_head(pb.BELLARD, 0x7F, 2 ** 61, 0, 2 ** 64 - 1, 64, None, 0,
                            ctypes.byref(count)) == pb.PI_EUNSUPPORTED
    # an empty range plans nothing
    assert pb.plan_head(pb.BELLARD, 10 ** 6, 96, 5, 5) == []


def test_instruction_model_uses_the_planners_class_cuts():
    # bench.py's per-term model splits each series at the same moduli as the
    # planner (fast arithmetic), so it prices every segment at its own class
    import bench
    firsts = [m for _, m, _, _, _, _, _ in bench.KERNEL_CLASSES]
    assert firsts == [0] + [2 ** lo for _, lo, _ in FAST[1:]]
    names = [name for name, *_ in bench.KERNEL_CLASSES]
    assert names == ["22", "27", "29", "f4", "f3", "f2", "fs", "62"]
    # and the model's head-term count is the planner's
    for f, n in ((pb.BELLARD, 10 ** 12), (pb.BBP, 10 ** 10), (pb.BELLARD, 2 * 10 ** 15)):
        ops, terms = bench.valu_ops_per_launch(f, n, 320)
        assert terms == pb.head_terms(f, n) and ops > 0
