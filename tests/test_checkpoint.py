"""Checkpoint bookkeeping (CPU): the pieces partition every series' index
range exactly, the file round-trips, a damaged piece is recomputed, a file
with a dropped, duplicated or overlapping piece is refused, and a corrupted
partial that passes every file check is caught by the n / n - 4 overlap."""
import copy
import json

import pytest

from paper_1008_3171_amd import checkpoint


def test_plan_partitions_each_series():
    ck = checkpoint.plan(1, 10 ** 9 + 1, 256, 320, 5)
    kmax = (10 ** 9 + 1 + 320) // 10 + 2
    for j in range(7):
        rs = sorted((it["k0"], it["k1"]) for it in ck["items"] if it["j"] == j)
        assert rs[0][0] == 0 and rs[-1][1] == kmax
        assert all(a[1] == b[0] for a, b in zip(rs, rs[1:]))
    assert len(checkpoint.plan(0, 1000, 8, 72, 3)["items"]) == 12


def test_roundtrip_and_damaged_piece_is_recomputed(tmp_path):
    path = str(tmp_path / "ck.json")
    ck = checkpoint.plan(1, 12345, 64, 128, 2)
    it = ck["items"][3]
    it["S"], it["N"], it["seconds"] = "1234abcd", 77, 0.1
    it["hash"] = checkpoint._digest(it)
    checkpoint.save(ck, path)
    back = checkpoint.load(path)
    assert back["items"][3]["S"] == "1234abcd" and 3 not in checkpoint.pending(back)
    raw = json.load(open(path))
    raw["items"][3]["S"] = "1234abce"                 # one flipped bit
    json.dump(raw, open(path, "w"))
    back = checkpoint.load(path)
    assert 3 in checkpoint.pending(back)


def test_dropped_duplicated_or_overlapping_pieces_fail_loudly(tmp_path):
    path = str(tmp_path / "ck.json")
    ck = checkpoint.plan(1, 10 ** 7 + 1, 256, 320, 4)
    checkpoint.validate(ck)
    bad = []
    dropped = copy.deepcopy(ck)
    del dropped["items"][5]
    bad.append(dropped)
    duplicated = copy.deepcopy(ck)
    duplicated["items"].append(copy.deepcopy(ck["items"][9]))
    bad.append(duplicated)
    overlapping = copy.deepcopy(ck)
    overlapping["items"][2]["k1"] += 1
    bad.append(overlapping)
    foreign = copy.deepcopy(ck)
    foreign["items"].append(dict(ck["items"][0], j=7))
    bad.append(foreign)
    for b in bad:
        checkpoint.save(b, path)
        with pytest.raises(ValueError):
            checkpoint.load(path)


def test_corrupted_partial_that_still_certifies_is_caught_by_the_n_minus_4_run(tmp_path):
    # A limb flipped high in a stored partial sum, with its hash rewritten to
    # match, passes every file check, and the guard window still certifies
    # (the flip is far above it): only the paper's double computation, at n
    # and n - 4, shows the bits are wrong.
    import oracle
    from paper_1008_3171_amd.verify import overlap
    from test_table_2_1_record import combine_on_cpu
    f, n, w, P = 1, 200_001, 64, 128
    L = (P + 63) // 64

    def record(pos):
        ck = checkpoint.plan(f, pos, w, P, 2)
        for it in ck["items"]:
            S, N = oracle.sum_slice(f, it["j"], pos - 1, it["k0"], it["k1"], P)
            it["S"], it["N"], it["seconds"] = "%x" % (S << (64 * L - P)), N, 0.0
            it["hash"] = checkpoint._digest(it)
        return ck

    good, lower = record(n), record(n - 4)
    bad = copy.deepcopy(good)
    it = bad["items"][3]
    it["S"] = "%x" % (int(it["S"], 16) ^ (1 << (64 * L - 20)))   # bit 20 of the result
    it["hash"] = checkpoint._digest(it)
    path = str(tmp_path / "bad.json")
    checkpoint.save(bad, path)
    bad = checkpoint.load(path)
    assert not checkpoint.pending(bad)                  # the file checks pass
    results = {}
    for name, ck in (("good", good), ("bad", bad), ("lower", lower)):
        S, N, cert = combine_on_cpu(ck)
        assert cert, name                               # all three certify
        results[name] = S >> (P - w)
    assert overlap(results["good"], results["lower"], w, 4)[2]
    assert not overlap(results["bad"], results["lower"], w, 4)[2]
