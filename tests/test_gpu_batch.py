"""pi_extract_batch: every query of a batch gives exactly what pi_extract_ex
gives alone (sum, N and certification), and what the oracle gives."""
import random

import pytest
import torch

import oracle
import paper_1008_3171_amd as pb
from paper_1008_3171_amd import workloads

pytestmark = pytest.mark.gpu


def run_batch(specs, with_workspace=False, with_status=True):
    qarr, total = pb.make_queries(specs)
    out = torch.zeros(max(1, total), dtype=torch.int64, device="cuda")
    status = torch.zeros(4 * max(1, len(specs)), dtype=torch.int32, device="cuda")
    ws = None
    if with_workspace:
        nbytes = pb.workspace_size(qarr, len(specs))
        ws = torch.zeros((nbytes + 7) // 8, dtype=torch.int64, device="cuda")
    pb.extract_batch(qarr, len(specs), out, status if with_status else False, workspace=ws)
    torch.cuda.synchronize()
    res = []
    vals = [int(v) & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
    for i, (f, n, w, P) in enumerate(specs):
        off = qarr[i].out_offset
        L = pb.limbs(P)
        S = 0
        for j in range(L):
            S |= vals[off + j] << (64 * j)
        S >>= 64 * L - P
        code, N = pb.status_of(status, i)
        res.append((S, N, code == pb.PI_OK))
    return res


def single(f, n, w, P):
    out, st = pb.extract(f, n, w, P)
    code, N = pb.status_of(st)
    return pb.to_int(out, P), N, code == pb.PI_OK


def test_mixed_small_batch_matches_single_and_oracle():
    rng = random.Random(77)
    specs = [(pb.BELLARD, 9, 8, 72), (pb.BBP, 1, 1, 1), (pb.BBP, 2, 64, 64)]
    for _ in range(120):
        f = rng.choice([pb.BBP, pb.BELLARD])
        n = rng.randrange(1, 200_000)
        P = rng.choice([64, 96, 128, 192, 320, 640, 1088, rng.randrange(1, 1089)])
        specs.append((f, n, rng.randrange(1, P + 1), P))
    specs.append(specs[5])                          # a duplicate query
    got = run_batch(specs)
    for spec, g in zip(specs, got):
        assert g == single(*spec), spec
        assert g == oracle.extract(*spec, 8), spec


def test_workspace_and_null_status():
    specs = workloads.batch_queries(64, seed=5, hi_exp=6)
    a = run_batch(specs, with_workspace=True)
    b = run_batch(specs, with_workspace=False)
    c = run_batch(specs, with_status=False)
    assert a == b
    assert [x[0] for x in a] == [x[0] for x in c]


def test_batch_of_4096_log_uniform_queries_equals_single_queries():
    # the benchmark's 4096-query batch (seed 1008): every result equals the
    # single-query call; a seeded sample of the small ones also the oracle's
    specs = workloads.batch_queries(4096, seed=1008)
    got = run_batch(specs)
    for spec, g in zip(specs, got):
        assert g == single(*spec), spec
        assert g[2], spec
    rng = random.Random(1008)
    small = [i for i, s in enumerate(specs) if s[1] <= 3_000_000]
    for i in rng.sample(small, 60):
        assert got[i] == oracle.extract(*specs[i], 8), specs[i]


def test_empty_and_invalid_batches():
    lib = pb.load()
    qarr, _ = pb.make_queries([])
    import ctypes
    assert lib.pi_extract_batch(ctypes.cast(qarr, ctypes.c_void_p), 0, None, None, None, 0,
                                None) == 0
    qarr, total = pb.make_queries([(pb.BELLARD, 1000, 8, 72), (pb.BELLARD, 0, 8, 72)])
    out = torch.zeros(total, dtype=torch.int64, device="cuda")
    with pytest.raises(pb.PiError):
        pb.extract_batch(qarr, 2, out)


def test_planned_batch_eager_and_graph_replays():
    # a batch plan launched eagerly equals pi_extract_batch; captured into a
    # HIP graph, every replay (with eager work in between) gives it again
    specs = workloads.batch_queries(256, seed=11, hi_exp=7)
    qarr, total = pb.make_queries(specs)
    ref = run_batch(specs)
    out = torch.zeros(total, dtype=torch.int64, device="cuda")
    status = torch.zeros(4 * len(specs), dtype=torch.int32, device="cuda")
    plan = pb.BatchPlan(qarr, len(specs), out, status)

    def results():
        vals = [int(v) & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
        res = []
        for i, (f, n, w, P) in enumerate(specs):
            L, off = pb.limbs(P), qarr[i].out_offset
            S = sum(vals[off + j] << (64 * j) for j in range(L)) >> (64 * L - P)
            code, N = pb.status_of(status, i)
            res.append((S, N, code == pb.PI_OK))
        return res

    plan.launch()
    torch.cuda.synchronize()
    assert results() == ref
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.launch(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(stream=torch.cuda.current_stream())
    for rep in range(3):
        out.zero_()
        status.zero_()
        single(pb.BELLARD, 10 ** 6 + rep, 64, 96)      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert results() == ref, rep
    plan.close()
