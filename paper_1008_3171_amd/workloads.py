"""Seeded synthetic workloads: the query streams the tests and the benchmark
feed to both the GPU library and the oracle.

This module only draws query parameters (formula, position, width,
precision, arrival times) from fixed seeds; it contains none of the
extraction arithmetic. Sizes follow the paper's workloads: positions spread
over decades as in Table 2.3 (10^9 .. 10^15), widths up to the 256 bits of
Table 2.1, and precision P = width + 64 guard bits.
"""
from __future__ import annotations

import numpy as np

BBP = 0
BELLARD = 1


def batch_queries(count: int = 4096, seed: int = 1008, lo_exp: float = 4.0,
                  hi_exp: float = 9.0, widths=(32, 64, 128, 256), formula: int = BELLARD):
    """[(formula, n, nbits, P)]: n = floor(10^U), U ~ Uniform(lo_exp, hi_exp),
    nbits uniform over `widths`, P = nbits + 64 (numpy PCG64 with `seed`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(lo_exp, hi_exp, size=count)
    w = rng.choice(np.asarray(widths), size=count)
    out = []
    for ui, wi in zip(u, w):
        n = max(1, int(10.0 ** float(ui)))
        out.append((formula, n, int(wi), int(wi) + 64))
    return out


def serving_stream(count: int = 20000, seed: int = 3171, lo_exp: float = 3.0,
                   hi_exp: float = 11.0, widths=(64, 256), rate: float = 1.0):
    """[(t_arrival, formula, n, nbits, P)]: Poisson arrivals at `rate` per
    second (exponential gaps), n = floor(10^U) with U ~ Uniform(lo_exp,
    hi_exp), formula BBP or Bellard with probability 1/2 each, nbits uniform
    over `widths`, P = nbits + 64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    u = rng.uniform(lo_exp, hi_exp, size=count)
    f = rng.integers(0, 2, size=count)
    w = rng.choice(np.asarray(widths), size=count)
    out = []
    for ti, ui, fi, wi in zip(t, u, f, w):
        n = max(1, int(10.0 ** float(ui)))
        out.append((float(ti), int(fi), n, int(wi), int(wi) + 64))
    return out
