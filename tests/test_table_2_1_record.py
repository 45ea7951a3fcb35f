"""The Table 2.1 checkpoint (records/table_2_1.json): n = 2*10^15 - 3, 256
bits, P = 320, split into per-series pieces computed on the GPU.

On the CPU: every piece's hash holds, the pieces of each series tile its
index range [0, (n + P) // 10 + 2) without gaps or overlaps, and every
finished piece's index count N equals its definition (every head index, plus
the tail indices before the first zero truncation). Once every piece is in,
the sum of the partial sums mod 2^P, certified against B = N + 2J, must give
the 256 bits the paper prints (Table 2.1), whose fourth is the title's 0."""
import json
import os

import pytest

from conftest import hex_bits, read_golden
from test_oracle_pins import boundary_certifies, n_definition_series

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORD = os.path.join(ROOT, "records", "table_2_1.json")


@pytest.fixture(scope="module")
def record():
    if not os.path.exists(RECORD):
        pytest.skip("no Table 2.1 record")
    from paper_1008_3171_amd import checkpoint
    raw = json.load(open(RECORD))
    ck = checkpoint.load(RECORD)           # a piece whose hash fails is reset to pending
    return raw, ck


def test_pieces_are_intact_and_tile_every_series(record):
    raw, ck = record
    (n, nbits, _), = read_golden("table_2_1.txt")
    assert (ck["formula"], ck["n"], ck["nbits"], ck["P"]) == (1, int(n), int(nbits), 320)
    for a, b in zip(raw["items"], ck["items"]):
        assert (a["S"] is None) == (b["S"] is None), a      # no finished piece lost its hash
    kmax = (ck["n"] + ck["P"]) // 10 + 2
    for j in range(7):
        items = sorted((it for it in ck["items"] if it["j"] == j), key=lambda it: it["k0"])
        assert items[0]["k0"] == 0 and items[-1]["k1"] == kmax
        for x, y in zip(items, items[1:]):
            assert x["k1"] == y["k0"]


def test_finished_pieces_count_their_indices(record):
    raw, ck = record
    done = [it for it in ck["items"] if it["S"] is not None]
    assert done
    d = ck["n"] - 1
    for it in done:
        want = n_definition_series(1, it["j"], d, ck["P"], it["k0"], it["k1"]) \
            if it["k1"] - it["k0"] < 10 ** 6 else None
        if want is None:
            # a long range: all head indices unless it reaches the tail
            from oracle import series_table
            rows, step, _ = series_table(1)
            K = (d + rows[it["j"]][1]) // step + 1
            head = max(0, min(it["k1"], K) - it["k0"])
            tail_from = max(it["k0"], K)
            tail = n_definition_series(1, it["j"], d, ck["P"], tail_from, it["k1"]) \
                if tail_from < it["k1"] else 0
            want = head + tail
        assert it["N"] == want, it


def combine_on_cpu(ck):
    """(S, N, certified) of a complete record: the pieces' left-aligned L-limb
    partial sums added mod 2^(64L), shifted down to P bits, and certified
    against B = N + 2J (J series)."""
    P, w = ck["P"], ck["nbits"]
    L = (P + 63) // 64
    total = sum(int(it["S"], 16) for it in ck["items"]) % 2 ** (64 * L)
    S = total >> (64 * L - P)
    N = sum(it["N"] for it in ck["items"])
    J = len({it["j"] for it in ck["items"]})
    return S, N, boundary_certifies(S, P, w, N + 2 * J)


def test_combination_on_a_small_record_filled_by_the_oracle(tmp_path):
    # the same completion path on a record whose pieces the oracle computed,
    # stored the way the GPU runner stores them (left-aligned limbs, hashed)
    import oracle
    from paper_1008_3171_amd import checkpoint
    for f, n, w, P, pieces in ((1, 10 ** 6 + 1, 256, 320, 3), (0, 54321, 64, 100, 4)):
        ck = checkpoint.plan(f, n, w, P, pieces)
        L = (P + 63) // 64
        for it in ck["items"]:
            S, N = oracle.sum_slice(f, it["j"], n - 1, it["k0"], it["k1"], P)
            it["S"], it["N"], it["seconds"] = "%x" % (S << (64 * L - P)), N, 0.0
            it["hash"] = checkpoint._digest(it)
        path = str(tmp_path / "ck.json")
        checkpoint.save(ck, path)
        back = checkpoint.load(path)
        assert not checkpoint.pending(back)
        S, N, cert = combine_on_cpu(back)
        assert (S, N, cert) == oracle.extract(f, n, w, P)


def test_complete_record_gives_table_2_1(record):
    raw, ck = record
    pending = [it for it in ck["items"] if it["S"] is None]
    if pending:
        pytest.skip("%d of %d pieces still to run" % (len(pending), len(ck["items"])))
    P, w = ck["P"], ck["nbits"]
    S, N, cert = combine_on_cpu(ck)
    assert cert
    (n, nbits, h), = read_golden("table_2_1.txt")
    assert int(n) == ck["n"] and S >> (P - w) == hex_bits(h, int(nbits))
    assert (S >> (P - 4)) & 1 == 0          # bit 2*10^15, the title's bit
