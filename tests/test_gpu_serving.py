"""The continuous-batching server: every query's result is bit-identical to
pi_extract_ex alone, whatever else is in flight; slots are admitted and
reused; a large query keeps its partial sum on the device across steps."""
import os
import random

import pytest

import oracle
import paper_1008_3171_amd as pb
from paper_1008_3171_amd import serving, workloads

pytestmark = pytest.mark.gpu


def alone(f, n, w, P):
    out, st = pb.extract(f, n, w, P)
    code, N = pb.status_of(st)
    return pb.to_int(out, P), code, N


def test_results_alone_equal_results_in_the_mix():
    stream = workloads.serving_stream(400, seed=3171, hi_exp=8.0, rate=4000.0)
    srv = pb.Server(max_active=48, step_terms=1 << 22)
    results, lat, makespan, steps = serving.run_stream(srv, stream)
    srv.close()
    assert len(results) == len(stream)
    assert steps > 10                       # the queries really overlapped
    for tag, (ta, f, n, w, P) in enumerate(stream):
        assert results[tag] == alone(f, n, w, P), (tag, f, n, w, P)
    rng = random.Random(3171)
    small = [t for t, q in enumerate(stream) if q[2] <= 2_000_000]
    for tag in rng.sample(small, 25):
        ta, f, n, w, P = stream[tag]
        S, N, cert = oracle.extract(f, n, w, P, 8)
        assert results[tag] == (S, 0 if cert else 1, N)


def test_unpipelined_steps_give_the_same_results():
    stream = workloads.serving_stream(120, seed=77, hi_exp=7.0, rate=2000.0)
    out = []
    for depth in (1, 0):
        srv = pb.Server(max_active=24, step_terms=1 << 21)
        srv.set_pipeline(depth)
        results, lat, makespan, steps = serving.run_stream(srv, stream)
        srv.close()
        assert len(results) == len(stream) and steps > 5
        out.append(results)
    assert out[0] == out[1]
    with pytest.raises(pb.PiError):
        pb.Server(max_active=2).set_pipeline(2)


def test_admission_busy_and_slot_reuse():
    srv = pb.Server(max_active=2, step_terms=1 << 20)
    assert srv.capacity() == 2
    assert srv.submit(pb.BELLARD, 10 ** 6, 64, 128, 1)
    assert srv.submit(pb.BBP, 12345, 256, 320, 2)
    assert not srv.submit(pb.BELLARD, 999, 8, 72, 3)        # no free slot
    got = {}
    while srv.active():
        srv.step()
        for tag, S, code, N in srv.poll():
            got[tag] = (S, code, N)
    assert srv.submit(pb.BELLARD, 999, 8, 72, 3)            # a slot came back
    while srv.active():
        srv.step()
        for tag, S, code, N in srv.poll():
            got[tag] = (S, code, N)
    srv.close()
    assert got[1] == alone(pb.BELLARD, 10 ** 6, 64, 128)
    assert got[2] == alone(pb.BBP, 12345, 256, 320)
    assert got[3] == alone(pb.BELLARD, 999, 8, 72)
    with pytest.raises(pb.PiError):
        pb.Server(max_active=4).submit(pb.BELLARD, 0, 8, 72, 0)


def test_large_query_spans_many_steps_while_small_ones_finish():
    srv = pb.Server(max_active=16, step_terms=1 << 24)
    big = (pb.BELLARD, 10 ** 9 + 1, 256, 320)
    assert srv.submit(*big, 0)
    steps = 0
    got = {}
    small = [(pb.BBP, 1000 + 7 * i, 64, 128) for i in range(40)]
    for i, q in enumerate(small):
        while not srv.submit(*q, i + 1):
            srv.step()
            steps += 1
            got.update({t: (S, c, N) for t, S, c, N in srv.poll()})
    while srv.active():
        srv.step()
        steps += 1
        got.update({t: (S, c, N) for t, S, c, N in srv.poll()})
    srv.close()
    assert steps > 20
    assert got[0] == alone(*big)
    for i, q in enumerate(small):
        assert got[i + 1] == alone(*q)


def test_paper_scale_slice_subslices_match_oracle():
    # n = 2*10^15, k in [10^14, 10^14 + 2^32): moduli near 2^50; seeded
    # 10^6-term sub-slices of it, every series, against the oracle
    n = 2 * 10 ** 15
    rng = random.Random(1008)
    for j in range(7):
        k0 = 10 ** 14 + rng.randrange(0, 2 ** 32 - 150_000)
        k1 = k0 + 142_858
        P = 320
        got = pb.to_int(pb.sum_slice(pb.term_id(pb.BELLARD, j), n, k0, k1, P), P)
        assert got == oracle.sum_slice(oracle.BELLARD, j, n - 1, k0, k1, P, 8)[0], (j, k0)


def test_server_in_a_process_that_loads_the_library_before_torch():
    # the library loaded first (a host-only call) and then a server as the
    # process's first GPU work: one HIP runtime, server creation works
    import subprocess
    import sys
    code = ("import paper_1008_3171_amd as pb\n"
            "assert pb.head_terms(pb.BELLARD, 10 ** 6) == 700001\n"
            "s = pb.Server(max_active=1024, step_terms=1 << 20)\n"
            "assert s.submit(pb.BELLARD, 9, 8, 72, 7)\n"
            "while s.active():\n"
            "    s.step()\n"
            "(tag, S, code, N), = s.poll()\n"
            "s.close()\n"
            "assert tag == 7 and code == pb.PI_OK and S >> 64 == 0x3F\n"
            "print('ok')\n")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert res.returncode == 0 and "ok" in res.stdout, res.stderr[-2000:]


def test_admission_by_device_memory():
    # the memory cap decides how many queries are admitted at once: find the
    # cap that allows three slots, fill them, see the fourth refused, and see
    # it admitted once a slot's query has finished
    srv = pb.Server(max_active=64, step_terms=1 << 20)
    srv.set_memory_limit(0)
    assert srv.capacity() == 0
    assert not srv.submit(pb.BELLARD, 999, 8, 72, 0)
    cap_bytes = None
    for kib in range(1, 1024):
        srv.set_memory_limit(kib * 1024)
        if srv.capacity() == 3:
            cap_bytes = kib * 1024
            break
    assert cap_bytes is not None
    qs = [(pb.BELLARD, 10 ** 6 + i, 64, 128) for i in range(3)] + [(pb.BBP, 4321, 256, 320)]
    for i, q in enumerate(qs[:3]):
        assert srv.submit(*q, i)
    assert not srv.submit(*qs[3], 3)
    got = {}
    while srv.active():
        srv.step()
        got.update({t: (S, c, N) for t, S, c, N in srv.poll()})
    assert srv.submit(*qs[3], 3)
    while srv.active():
        srv.step()
        got.update({t: (S, c, N) for t, S, c, N in srv.poll()})
    srv.close()
    for i, q in enumerate(qs):
        assert got[i] == alone(*q), (i, q)


def test_slot_pool_grows_on_demand():
    # more queries at once than the pool's first allocation: it doubles as
    # admission needs slots, and every result still equals the query alone
    stream = workloads.serving_stream(300, seed=1008, hi_exp=7.0, rate=1e9)
    srv = pb.Server(max_active=300, step_terms=1 << 22)
    assert srv.capacity() == 300
    for tag, (ta, f, n, w, P) in enumerate(stream):
        assert srv.submit(f, n, w, P, tag)
    assert srv.active() == 300
    got = {}
    steps = 0
    while srv.active():
        srv.step()
        steps += 1
        got.update({t: (S, c, N) for t, S, c, N in srv.poll()})
    srv.close()
    assert len(got) == 300 and steps > 1
    for tag, (ta, f, n, w, P) in enumerate(stream):
        assert got[tag] == alone(f, n, w, P), (tag, f, n, w, P)


def test_steps_mixing_fused_and_wide_queries():
    # queries of 1 to 6 limbs share a step's fused launch; wider ones (8, 12,
    # 17 limbs) get their own launches in the same step; every result equals
    # the query alone
    rng = random.Random(4242)
    qs = []
    for i in range(36):
        P = rng.choice([64, 96, 192, 320, 384, 448, 640, 1024, 1088])
        qs.append((rng.choice([pb.BBP, pb.BELLARD]), rng.randrange(1, 3_000_000),
                   rng.randrange(1, P + 1), P))
    for depth in (1, 0):
        srv = pb.Server(max_active=12, step_terms=1 << 20)
        srv.set_pipeline(depth)
        got, i, steps = {}, 0, 0
        while i < len(qs) or srv.active():
            while i < len(qs) and srv.submit(*qs[i], i):
                i += 1
            srv.step()
            steps += 1
            got.update({t: (S, c, N) for t, S, c, N in srv.poll()})
        srv.close()
        assert steps > 3 and len(got) == len(qs)
        for t, q in enumerate(qs):
            assert got[t] == alone(*q), (depth, t, q)
