"""Checkpointed extraction (partial sums persisted between calls, summed and
certified on the device) equals the one-call extraction bit for bit; slice
counts N equal the oracle's."""
import random
import sys

import pytest

import oracle
import paper_1008_3171_amd as pb
from conftest import hex_bits, read_golden
from test_oracle_pins import n_definition
from paper_1008_3171_amd import checkpoint

pytestmark = pytest.mark.gpu


def alone(f, n, w, P):
    out, st = pb.extract(f, n, w, P)
    code, N = pb.status_of(st)
    return pb.to_int(out, P), code, N


def test_slice_counts_match_oracle():
    rng = random.Random(8)
    for f in (pb.BBP, pb.BELLARD):
        for j in range(4 if f == pb.BBP else 7):
            n = rng.randrange(1, 10 ** 6)
            P = rng.choice([64, 320])
            kmax = (n + P) // (4 if f == pb.BBP else 10) + 2
            k0 = rng.randrange(0, kmax)
            k1 = rng.randrange(k0, kmax + 50)
            out, st = pb.sum_slice_ex(pb.term_id(f, j), n, k0, k1, P)
            S, N = oracle.sum_slice(f, j, n - 1, k0, k1, P, 8)
            assert (pb.to_int(out, P), pb.status_of(st)) == (S, (0, N))


def test_interrupted_and_resumed_extraction_equals_one_call(tmp_path):
    path = str(tmp_path / "ck.json")
    for f, n, w, P in ((pb.BELLARD, 10 ** 8 + 1, 256, 320), (pb.BBP, 7654321, 64, 96)):
        ck = checkpoint.plan(f, n, w, P, 3)
        checkpoint.save(ck, path)
        assert checkpoint.run(checkpoint.load(path), path, 1e9, max_pieces=5) == 5
        ck = checkpoint.load(path)                       # "a later process" resumes
        assert len(checkpoint.pending(ck)) == len(ck["items"]) - 5
        checkpoint.run(ck, path, 1e9)
        assert checkpoint.finish(checkpoint.load(path)) == alone(f, n, w, P)


def test_combine_certifies_like_extract():
    # an uncertain case: too few guard bits for N
    f, n, w, P = pb.BELLARD, 100_001, 60, 64
    ck = checkpoint.plan(f, n, w, P, 2)
    checkpoint.run(ck, None, 1e9)
    got = checkpoint.finish(ck)
    assert got == alone(f, n, w, P)
    assert got[1] == pb.PI_UNCERTAIN


@pytest.mark.timeout(600)
def test_table_2_2_row_m13_checkpointed(tmp_path):
    # n = 10^13 + 1: 7.0e12 head terms, about 71 s on one MI355X at P = 1088, in
    # 28 checkpointed pieces; every printed bit (1000) must equal the row,
    # certified, with N equal to its definition
    row = [r for r in read_golden("table_2_2.txt") if r[0] == "13"][0]
    n, nbits = int(row[1]), int(row[2])
    P = 1088
    ck = checkpoint.plan(pb.BELLARD, n, nbits, P, 4)
    path = str(tmp_path / "m13.json")
    checkpoint.save(ck, path)
    checkpoint.run(checkpoint.load(path), path, 1e9, log=sys.stdout)
    ck = checkpoint.load(path)
    S, code, N = checkpoint.finish(ck)
    assert N == n_definition(pb.BELLARD, n - 1, P)
    assert code == pb.PI_OK
    assert S >> (P - nbits) == hex_bits(row[3], nbits)


def test_double_run_overlap():
    from paper_1008_3171_amd import verify
    row = [r for r in read_golden("table_2_2.txt") if r[0] == "11"][0]
    bits, count, agree = verify.double_run(pb.BELLARD, int(row[1]) + 4, 256)
    assert agree and count == 252
    # the overlap starts at 10^11 + 5: bits 4.. of the printed row
    assert bits == (hex_bits(row[3], 256) & ((1 << 252) - 1))
