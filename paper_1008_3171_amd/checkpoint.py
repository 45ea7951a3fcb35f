"""Interruptible, resumable extraction (section 4: the partial sums of jobs
are persisted, so a long computation can be stopped and resumed).

A checkpoint is a JSON file listing the pieces of one extraction: per series,
a partition of the index range [0, (n + P) // step + 2) (every head index and
every nonzero tail index) into `pieces` ranges. `run` computes pending pieces
with pi_sum_slice_ex, one at a time, and rewrites the file after each; a
piece stores its partial sum S, its index count N and a hash of both, and a
piece whose hash does not match is computed again, and a file whose pieces do
not tile every series' range exactly once is refused. `finish` adds the
partial sums on the device with pi_combine and certifies the total.

    python -m paper_1008_3171_amd.checkpoint plan  FILE --formula bellard --n N --nbits W --P P --pieces K
    python -m paper_1008_3171_amd.checkpoint run   FILE --budget SECONDS
    python -m paper_1008_3171_amd.checkpoint finish FILE
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

FORMULAS = {"bbp": 0, "bellard": 1}
STEP = {0: 4, 1: 10}
NSERIES = {0: 4, 1: 7}


def _digest(item) -> str:
    key = "%d:%d:%d:%s:%d" % (item["j"], item["k0"], item["k1"], item["S"], item["N"])
    return hashlib.sha256(key.encode()).hexdigest()


def plan(formula: int, n: int, nbits: int, P: int, pieces: int) -> dict:
    kmax = (n + P) // STEP[formula] + 2
    items = []
    for j in range(NSERIES[formula]):
        for p in range(pieces):
            items.append({"j": j, "k0": kmax * p // pieces, "k1": kmax * (p + 1) // pieces,
                          "S": None, "N": None, "hash": None, "seconds": None})
    return {"formula": formula, "n": n, "nbits": nbits, "P": P, "items": items}


def validate(ck: dict) -> None:
    """Every series of the formula must have pieces that tile its index range
    [0, (n + P) // step + 2) exactly once: a piece dropped, duplicated or
    overlapping would silently change the sum, so it raises ValueError."""
    f = ck["formula"]
    kmax = (ck["n"] + ck["P"]) // STEP[f] + 2
    for j in range(NSERIES[f]):
        rs = sorted((it["k0"], it["k1"]) for it in ck["items"] if it["j"] == j)
        if not rs or rs[0][0] != 0 or rs[-1][1] != kmax:
            raise ValueError("series %d does not cover [0, %d)" % (j, kmax))
        for a, b in zip(rs, rs[1:]):
            if a[1] != b[0]:
                raise ValueError("series %d: pieces [%d, %d) and [%d, %d) leave a gap or overlap"
                                 % (j, a[0], a[1], b[0], b[1]))
    if any(not 0 <= it["j"] < NSERIES[f] for it in ck["items"]):
        raise ValueError("a piece names a series the formula does not have")


def load(path: str) -> dict:
    with open(path) as f:
        ck = json.load(f)
    validate(ck)
    for it in ck["items"]:
        if it["S"] is not None and it["hash"] != _digest(it):
            it["S"] = it["N"] = it["hash"] = None          # damaged: compute again
    return ck


def save(ck: dict, path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(ck, f, indent=1)
    os.replace(tmp, path)


def pending(ck: dict):
    return [i for i, it in enumerate(ck["items"]) if it["S"] is None]


def run(ck: dict, path: str | None, budget_s: float, log=None, max_pieces=None) -> int:
    """Compute pending pieces until none is left, budget_s has passed or
    max_pieces were computed."""
    import torch
    import paper_1008_3171_amd as pb
    t0 = time.perf_counter()
    done = 0
    for i in pending(ck):
        if time.perf_counter() - t0 >= budget_s or (max_pieces is not None and done >= max_pieces):
            break
        it = ck["items"][i]
        t1 = time.perf_counter()
        out, st = pb.sum_slice_ex(pb.term_id(ck["formula"], it["j"]), ck["n"], it["k0"],
                                  it["k1"], ck["P"])
        torch.cuda.synchronize()
        it["S"] = "%x" % pb.to_int(out)              # the left-aligned limbs, as one integer
        it["N"] = pb.status_of(st)[1]
        it["seconds"] = time.perf_counter() - t1
        it["hash"] = _digest(it)
        done += 1
        if path:
            save(ck, path)
        if log:
            print("piece %d/%d (series %d, k %d..%d) %.1f s" % (
                i + 1, len(ck["items"]), it["j"], it["k0"], it["k1"], it["seconds"]),
                file=log, flush=True)
    return done


def finish(ck: dict):
    """(S, code, N): the P-bit sum, PI_OK/PI_UNCERTAIN and the index count."""
    import torch
    import paper_1008_3171_amd as pb
    if pending(ck):
        raise RuntimeError("%d pieces still pending" % len(pending(ck)))
    P = ck["P"]
    L = pb.limbs(P)
    words = []
    for it in ck["items"]:
        v = int(it["S"], 16)
        for i in range(L):
            w = (v >> (64 * i)) & 0xFFFFFFFFFFFFFFFF
            words.append(w - (1 << 64) if w >= 1 << 63 else w)
    parts = torch.tensor(words, dtype=torch.int64, device="cuda")
    N = sum(it["N"] for it in ck["items"])
    out, st = pb.combine(parts, len(ck["items"]), P, ck["nbits"], NSERIES[ck["formula"]], N)
    torch.cuda.synchronize()
    code, n_out = pb.status_of(st)
    return pb.to_int(out, P), code, n_out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("cmd", choices=["plan", "run", "finish"])
    ap.add_argument("file")
    ap.add_argument("--formula", choices=sorted(FORMULAS), default="bellard")
    ap.add_argument("--n", type=int)
    ap.add_argument("--nbits", type=int, default=256)
    ap.add_argument("--P", type=int, default=320)
    ap.add_argument("--pieces", type=int, default=8)
    ap.add_argument("--budget", type=float, default=600.0)
    args = ap.parse_args(argv)
    if args.cmd == "plan":
        save(plan(FORMULAS[args.formula], args.n, args.nbits, args.P, args.pieces), args.file)
        return 0
    ck = load(args.file)
    if args.cmd == "run":
        run(ck, args.file, args.budget, log=sys.stdout)
        print("pending pieces: %d" % len(pending(ck)), flush=True)
        return 0
    S, code, N = finish(ck)
    w, P = ck["nbits"], ck["P"]
    print(json.dumps({"n": ck["n"], "nbits": w, "P": P, "certified": code == 0, "N": N,
                      "hex": "%0*X" % ((w + 3) // 4, S >> (P - w)),
                      "gpu_seconds": sum(it["seconds"] for it in ck["items"])}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
