"""Exactness of the head kernel's binary64 arithmetic, checked on the CPU.

The GPU parity tests compare whole sums with the oracle. These tests pin the
arithmetic design itself at its worst cases, where random positions rarely
land:
- residues at the edge of each class's invariant;
- the largest window digit;
- moduli at both ends of each class;
- a reciprocal taken by one Newton step from the previous modulus.

`binary64_ladder.c` models the kernel's step with the C library's correctly
rounded fma. Every result must equal 2^d x^2 mod M exactly, with both
intermediate values below 2^53 and the result inside the invariant. The
32-bit-digit Hensel division is checked by its recurrence in Python integers.
"""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

# (window bits W, lowest modulus, first modulus past the class, second
# reduction, Newton steps per modulus)
CLASSES = [(4, 2 ** 29, 2 ** 33, False, 2), (3, 2 ** 33, 2 ** 42, False, 1),
           (2, 2 ** 42, 2 ** 46, False, 1), (1, 2 ** 46, 2 ** 48, False, 1),
           (2, 2 ** 48, 2 ** 51, True, 1)]


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("b64") / "binary64_ladder")
    subprocess.run(["gcc", "-O2", "-o", exe, os.path.join(HERE, "binary64_ladder.c"), "-lm"],
                   check=True)

    def run(lines):
        res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True,
                             text=True, check=True)
        return res.stdout.split("\n")[:len(lines)]
    return run


def edge_moduli(lo, hi, rng):
    ms = [lo + 1, lo + 3, hi - 1, hi - 3, hi - 21]
    ms += [rng.randrange(lo, hi) | 1 for _ in range(6)]
    ms += [rng.randrange(hi - hi // 64, hi) | 1 for _ in range(6)]
    return ms


@pytest.mark.parametrize("W,lo,hi,re,steps", CLASSES)
def test_step_is_exact_at_the_edges(model, W, lo, hi, re, steps):
    rng = random.Random(W * 100 + hi.bit_length())
    cases = []
    for M in edge_moduli(lo, hi, rng):
        bound = M // 2 + 1 if re else M - 1  # the class's residue invariant
        xs = [bound, -bound, bound - 1, -(bound - 7), 1, -1] + \
             [rng.randrange(-bound, bound + 1) for _ in range(12)]
        for x in xs:
            for d in {0, 1, (1 << W) - 1}:
                for mode in (0, steps):
                    cases.append((M, d, x, mode))
    out = model(["S %d %d %d %d %d" % (M, d, x, int(re), mode) for M, d, x, mode in cases])
    for (M, d, x, mode), line in zip(cases, out):
        y, ok = (int(v) for v in line.split())
        assert ok == 1, (M, d, x, mode)
        assert (y - (x * x << d)) % M == 0, (M, d, x, mode)
        assert abs(y) < M
        if re:
            assert abs(y) <= M // 2 + 1


@pytest.mark.parametrize("W,lo,hi,re,steps", CLASSES)
def test_ladder_equals_pow(model, W, lo, hi, re, steps):
    rng = random.Random(7 + W + hi.bit_length())
    cases = []
    for M in edge_moduli(lo, hi, rng):
        for _ in range(20):
            X = rng.getrandbits(rng.randrange(1, 62)) | 1
            cases.append((M, X))
        cases += [(M, 1), (M, 63), (M, 64), (M, 2 ** 61 - 1), (M, 2 ** 61 + 12345)]
    out = model(["L %d %d %d %d %d" % (M, X, W, int(re), steps) for M, X in cases])
    for (M, X), line in zip(cases, out):
        assert int(line) == pow(2, X, M), (M, X, W, re)


def test_hensel_digit_recurrence():
    # h' = (u m1 + (u m0 + h) / 2^31) / 2 with u = lo32(h) * (-M^-1 mod 2^32)
    # and M = m1 2^31 + m0: no intermediate reaches 2^64, h stays below M, and
    # the digits are -s M^-1 mod 2^(64L)
    rng = random.Random(3171)
    for _ in range(3000):
        bits = rng.choice([31, 32, 40, 42, 46, 48, 51, 54])
        M = rng.getrandbits(bits) | 1 | (1 << (bits - 1))
        s = rng.choice([0, 1, M - 1, rng.randrange(M)])
        L = rng.choice([1, 2, 5, 17])
        mp = (-pow(M, -1, 2 ** 32)) % 2 ** 32
        m0, m1 = M & (2 ** 31 - 1), M >> 31
        h, t = s, 0
        for i in range(2 * L):
            u = ((h & 0xffffffff) * mp) & 0xffffffff
            A = u * m0 + h
            assert A < 2 ** 64 and A % 2 ** 31 == 0
            B = u * m1 + (A >> 31)
            assert B < 2 ** 64 and B % 2 == 0
            h = B >> 1
            assert h < M
            t |= u << (32 * i)
        assert t == (-s * pow(M, -1, 2 ** (64 * L))) % 2 ** (64 * L)
