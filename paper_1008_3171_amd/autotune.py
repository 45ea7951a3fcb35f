"""Autotuner for the head kernel's launch shapes.

Two kinds of launch are tuned, each on a workload of its own kind:

* the fused launch that batches and serving steps use for every query of 1
  to 6 limbs, on the seeded 4096-query batch itself (Bellard,
  n = floor(10^U) with U ~ U(4, 9), 32 to 256 result bits), timed as one
  pi_extract_batch call;
* the single-query instances of 2, 3 and 5 limbs, each on one extraction
  large enough (tenths of a second) that launch cost does not decide.

For each it times every candidate (workgroups per CU, run cap) and keeps the
fastest; results do not depend on the shape, which is checked (every
candidate's output must equal the default's). The choices are written as
JSON (by default into the package, where the binding applies them when the
library is loaded; PIBBP_TUNING names another file).

    python -m paper_1008_3171_amd.autotune [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

# limb class -> (formula, n, nbits, P): a single query of that class
SINGLE = {
    2: (1, 10 ** 10, 64, 128),
    3: (1, 10 ** 10, 128, 192),
    5: (1, 10 ** 11, 256, 320),
}
SINGLE_WG = (0, 4, 8)
SINGLE_CAPS = (256, 1024, 2048, 4096)
FUSED_WG = (0, 4, 5, 8)
FUSED_CAPS = (64, 256, 1024, 2048)
BATCH = dict(count=4096, seed=1008)
DEFAULT_CAP = 2048        # the library's run cap when nothing is tuned


def _timer(torch, stream, fn, reps):
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def single_runner(pb, torch, spec):
    f, n, w, P = spec
    out = torch.zeros(pb.limbs(P), dtype=torch.int64, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(reps=2):
        ms = _timer(torch, stream, lambda: pb.extract(f, n, w, P, out=out, status=st,
                                                      stream=stream), reps)
        return ms, (pb.to_int(out), pb.status_of(st))
    return run


def batch_runner(pb, torch):
    from paper_1008_3171_amd import workloads
    specs = workloads.batch_queries(BATCH["count"], seed=BATCH["seed"])
    qarr, total = pb.make_queries(specs)
    out = torch.zeros(total, dtype=torch.int64, device="cuda")
    st = torch.zeros(4 * len(specs), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(reps=2):
        ms = _timer(torch, stream, lambda: pb.extract_batch(qarr, len(specs), out, st,
                                                            stream=stream), reps)
        return ms, (out.cpu().tolist(), st.cpu().tolist())
    return run


def sweep(pb, key, runner, wgs, caps, log):
    default = pb.get_tuning(key)
    pb.set_tuning(key, 0, DEFAULT_CAP)
    runner()                                       # warm up
    base_ms, ref = runner()
    best = (base_ms, 0, DEFAULT_CAP)
    for wg in wgs:
        for cap in caps:
            pb.set_tuning(key, wg, cap)
            ms, val = runner()
            if val != ref:
                pb.set_tuning(key, *default)
                raise RuntimeError("launch shape changed the result: %r" % ((key, wg, cap),))
            print(json.dumps({"key": key, "wg_per_cu": wg, "run_cap": cap, "ms": ms}),
                  file=log, flush=True)
            if ms < best[0]:
                best = (ms, wg, cap)
    pb.set_tuning(key, best[1], best[2])
    return {"wg_per_cu": best[1], "run_cap": best[2], "ms": best[0], "default_ms": base_ms}


def tune(log=sys.stdout):
    import torch
    import paper_1008_3171_amd as pb
    arch = torch.cuda.get_device_properties(0).gcnArchName
    result = {"arch": arch, "classes": {}, "fused": None}
    for L in sorted(SINGLE):
        r = sweep(pb, L, single_runner(pb, torch, SINGLE[L]), SINGLE_WG, SINGLE_CAPS, log)
        r["workload"] = list(SINGLE[L])
        result["classes"][str(L)] = r
    r = sweep(pb, pb.TUNE_FUSED, batch_runner(pb, torch), FUSED_WG, FUSED_CAPS, log)
    r["workload"] = "pi_extract_batch of %d queries, seed %d" % (BATCH["count"], BATCH["seed"])
    result["fused"] = r
    return result


def main(argv=None):
    import paper_1008_3171_amd as pb
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None, help="cache file (default: the binding's)")
    args = ap.parse_args(argv)
    res = tune()
    path = args.out or pb.tuning_cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
