"""The paper's double computation (sections 2 and 3.1): extract at n and at
n - shift (usually 4) and accept only the bits both runs certify and agree
on; a disagreement points at a machine or transmission error.

    python -m paper_1008_3171_amd.verify --n N --nbits W [--P P] [--shift 4] [--formula bellard]
"""
from __future__ import annotations

import argparse
import json
import sys


def overlap(a: int, b: int, nbits: int, shift: int):
    """a: the nbits bits from position n; b: the nbits bits from n - shift.
    Returns (bits, count, agree): bits n .. n - shift + nbits - 1 as taken
    from a, their count, and whether b holds the same bits there."""
    count = nbits - shift
    a_head = a >> shift                              # bits n .. n + count - 1
    b_tail = b & ((1 << count) - 1)                  # the same positions from the second run
    return a_head, count, a_head == b_tail


def double_run(formula: int, n: int, nbits: int, P: int | None = None, shift: int = 4):
    """Returns (bits, count, agree): the overlap bits [n, n - shift + nbits) as
    an integer of `count` bits, and whether the two runs agree on them. Both
    runs must be certified, else ValueError."""
    import torch
    import paper_1008_3171_amd as pb
    if not 0 < shift < nbits or shift >= n:
        raise ValueError("need 0 < shift < nbits and shift < n")
    P = nbits + 64 if P is None else P
    a_out, a_st = pb.extract(formula, n, nbits, P)
    b_out, b_st = pb.extract(formula, n - shift, nbits, P)
    torch.cuda.synchronize()
    if pb.status_of(a_st)[0] != pb.PI_OK or pb.status_of(b_st)[0] != pb.PI_OK:
        raise ValueError("a run is not certified; use a larger P")
    a = pb.to_int(a_out, P) >> (P - nbits)          # bits n .. n + nbits - 1
    b = pb.to_int(b_out, P) >> (P - nbits)          # bits n - shift .. n - shift + nbits - 1
    return overlap(a, b, nbits, shift)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--nbits", type=int, default=256)
    ap.add_argument("--P", type=int)
    ap.add_argument("--shift", type=int, default=4)
    ap.add_argument("--formula", choices=["bbp", "bellard"], default="bellard")
    args = ap.parse_args(argv)
    f = 1 if args.formula == "bellard" else 0
    bits, count, agree = double_run(f, args.n, args.nbits, args.P, args.shift)
    print(json.dumps({"n": args.n, "bits": count, "agree": agree,
                      "hex": "%0*X" % ((count + 3) // 4, bits << ((-count) % 4))}))
    return 0 if agree else 1


if __name__ == "__main__":
    sys.exit(main())
