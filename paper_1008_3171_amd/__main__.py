"""Extract bits of pi on the GPU from the command line.

    python -m paper_1008_3171_amd --n 1000000000001 --nbits 256
    python -m paper_1008_3171_amd --n 9 --nbits 8 --formula bbp

Prints one JSON line: the bits in hex, whether the guard bits certify them
(section 3.1), the number of terms summed and the GPU time. Long runs can be
split and resumed with `python -m paper_1008_3171_amd.checkpoint`.
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1008_3171_amd",
                                 description="nbits bits of pi from 1-based position n")
    ap.add_argument("--n", type=int, required=True, help="position of the first bit (1-based)")
    ap.add_argument("--nbits", type=int, default=64)
    ap.add_argument("--P", type=int, default=0, help="working precision (default nbits + 64)")
    ap.add_argument("--formula", choices=["bellard", "bbp"], default="bellard")
    args = ap.parse_args(argv)

    import torch
    import paper_1008_3171_amd as pb

    formula = pb.BELLARD if args.formula == "bellard" else pb.BBP
    P = args.P or args.nbits + 64
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    out, st = pb.extract(formula, args.n, args.nbits, P, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    S = pb.to_int(out, P)
    code, N = pb.status_of(st)
    bits = S >> (P - args.nbits)
    print(json.dumps({"formula": args.formula, "n": args.n, "nbits": args.nbits, "P": P,
                      "hex": "%0*X" % ((args.nbits + 3) // 4, bits << ((-args.nbits) % 4)),
                      "certified": code == pb.PI_OK, "nterms": N,
                      "gpu_seconds": e0.elapsed_time(e1) * 1e-3}))
    return 0 if code == pb.PI_OK else 1


if __name__ == "__main__":
    sys.exit(main())
