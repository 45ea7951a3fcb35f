"""Seeded random slices against the oracle, bit for bit.

Each case draws a formula, a series, a position n (log-uniform up to 2^61),
a k range and a precision P. Half the ranges straddle a modulus-class cut of
the head kernel, a fifth sit at the head/tail boundary and the rest anywhere
in the head. Ranges past the 2^54 modulus limit are clipped to it.
"""
import random

import pytest

import oracle
import paper_1008_3171_amd as pb

pytestmark = pytest.mark.gpu

CUTS = [2 ** 22, 2 ** 27, 2 ** 29, 2 ** 31, 2 ** 33, 2 ** 36, 2 ** 42, 2 ** 46, 2 ** 48,
        2 ** 51, 2 ** 54]


def draw(rng):
    f = rng.choice([pb.BBP, pb.BELLARD])
    rows, step, _ = oracle.series_table(f)
    j = rng.randrange(len(rows))
    s, c, a, b = rows[j]
    n = int(2 ** rng.uniform(0, 61))
    K = max(0, (n - 1 + c) // step + 1)
    kmax = (2 ** 54 - 1 - b) // a + 1
    mode = rng.random()
    if mode < 0.5:
        cut = rng.choice(CUTS)
        kc = max(0, (cut - b + a - 1) // a)
        lo = step * (kc + 3000) + 10
        if lo < 2 ** 61:
            n = max(lo, int(2 ** rng.uniform(lo.bit_length(), 61.5)))
        k0 = max(0, kc - rng.randrange(0, 3000))
    elif mode < 0.7 and K > 0:
        k0 = max(0, K - rng.randrange(0, 3000))
    else:
        k0 = rng.randrange(0, max(1, min(K + 100, kmax)))
    k1 = min(k0 + rng.randrange(0, 6000), kmax)
    k0 = min(k0, k1)
    P = rng.choice([64, 96, 128, 320, 1088, rng.randrange(1, 1089)])
    return f, j, n, k0, k1, P


@pytest.mark.parametrize("seed", [1008, 3171])
def test_random_slices_equal_the_oracle(seed):
    rng = random.Random(seed)
    for _ in range(800):
        f, j, n, k0, k1, P = draw(rng)
        got = pb.to_int(pb.sum_slice(pb.term_id(f, j), n, k0, k1, P), P)
        assert got == oracle.sum_slice(f, j, n - 1, k0, k1, P, 8)[0], (f, j, n, k0, k1, P)
