"""Exactness of the head kernel's binary64 arithmetic, checked on the CPU.

The GPU parity tests compare whole sums with the oracle. These tests pin the
arithmetic design itself at its worst cases, where random positions rarely
land:
- residues at the edge of each class's invariant, through whole windows;
- every window digit;
- moduli at both ends of each class;
- a reciprocal taken by Newton steps from the previous modulus.

`binary64_ladder.c` models the kernel's step with the C library's correctly
rounded fma. Every window must give x^(2^W) 2^d mod M exactly, with every
intermediate value below 2^53 and the result inside the invariant. The
binary64 long division that turns a residue into its P-bit term must give
floor((x mod M) 2^P / M) mod 2^P from its signed digits, inside the digit
bounds that keep a run's per-position sums exact. The 32-bit-digit Hensel
division (integer classes) is checked by its recurrence in Python integers.
"""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

# (window bits W, lowest modulus, first modulus past the class, how a window
# applies its digit, Newton steps per modulus, invariant: |x| <= c M between
# windows). Digit modes: 0, in the window's last squaring; 2, after W plain
# squarings as its own scale-and-reduce step, which leaves |x| <= M/2 + M/2^20.
CLASSES = [(4, 2 ** 29, 2 ** 33, 0, 2, 1.0), (3, 2 ** 33, 2 ** 42, 0, 1, 1.0),
           (2, 2 ** 42, 2 ** 48, 0, 1, 0.75), (5, 2 ** 48, 2 ** 51, 2, 1, 0.5)]


def invariant(M, re, c):
    if re == 2:
        return M // 2 + (M >> 20)
    return min(int(c * M), M - 1)


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


@pytest.mark.parametrize("W,lo,hi,re,steps,c", CLASSES)
def test_window_keeps_the_invariant(model, W, lo, hi, re, steps, c):
    # one window from the edge of the invariant, with every digit: exact, the
    # right residue, and back inside the invariant
    rng = random.Random(W * 100 + hi.bit_length())
    cases = []
    for M in edge_moduli(lo, hi, rng):
        bound = invariant(M, re, c)
        xs = [bound, -bound, bound - 1, -(bound - 7), 1, -1] + \
             [rng.randrange(-bound, bound + 1) for _ in range(8)]
        for x in xs:
            for d in range(1 << W):
                for mode in (0, steps):
                    cases.append((M, d, x, mode))
    out = model(["W %d %d %d %d %d %d" % (M, W, d, x, re, mode) for M, d, x, mode in cases])
    for (M, d, x, mode), line in zip(cases, out):
        y, ok = (int(v) for v in line.split())
        assert ok == 1, (M, d, x, mode)
        assert (y - (pow(x, 2 ** W, M) << d)) % M == 0, (M, d, x, mode)
        assert abs(y) <= invariant(M, re, c), (M, d, x, y)


@pytest.mark.parametrize("W,lo,hi,re,steps,c", CLASSES)
def test_ladder_equals_pow(model, W, lo, hi, re, steps, c):
    rng = random.Random(7 + W + hi.bit_length())
    cases = []
    for M in edge_moduli(lo, hi, rng):
        for _ in range(20):
            X = rng.getrandbits(rng.randrange(1, 62)) | 1
            cases.append((M, X))
        cases += [(M, 1), (M, 63), (M, 64), (M, 2 ** 61 - 1), (M, 2 ** 61 + 12345)]
    out = model(["L %d %d %d %d %d" % (M, X, W, re, steps) for M, X in cases])
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



def test_hensel32_digit_recurrence():
    # 32-bit-digit Hensel division for moduli below 2^31: u = h * (-M^-1 mod
    # 2^32) mod 2^32, then h' = (h + uM) / 2^32 from one 64-bit multiply-add:
    # h + uM stays below 2^63, is divisible by 2^32, and h' stays below M;
    # the digits are -s M^-1 mod 2^(64L)
    rng = random.Random(32)
    for _ in range(3000):
        bits = rng.choice([2, 3, 20, 22, 27, 29, 30, 31])
        M = rng.getrandbits(bits) | 1 | (1 << (bits - 1))
        s = rng.choice([0, 1, M - 1, rng.randrange(M)])
        L = rng.choice([1, 2, 3, 5, 17])
        mp = (-pow(M, -1, 2 ** 32)) % 2 ** 32
        h, t = s, 0
        for i in range(2 * L):
            u = (h * mp) % 2 ** 32
            A = h + u * M
            assert A < 2 ** 63 and A % 2 ** 32 == 0
            h = A >> 32
            assert h < M
            t |= u << (32 * i)
        assert t == (-s * pow(M, -1, 2 ** (64 * L))) % 2 ** (64 * L)

# limb counts the kernels are built for; a query of P bits uses the smallest
# that holds it
LIMB_CLASSES = [1, 2, 3, 4, 5, 6, 8, 12, 17]


CARRY_TERMS = 120    # terms whose digits a lane sums between carry steps


def digit_layout(P):
    # the kernel's digit plan: as few digits as cover 64L bits, at most 46 bits
    L = next(c for c in LIMB_CLASSES if 64 * c >= P)
    N = -(-64 * L // 46)
    return N, -(-64 * L // N)


@pytest.mark.parametrize("W,lo,hi,re,steps,c", CLASSES)
def test_long_division_gives_the_truncated_term(model, W, lo, hi, re, steps, c):
    # x 2^P / M in signed digits: sum q_d 2^(dB) - [last remainder < 0] is
    # floor((x mod M) 2^P / M) mod 2^P for residues anywhere in the ladder's
    # invariant (negative ones included) and every limb class, with digits
    # small enough that CARRY_TERMS of them, added to a carried sum below
    # 2^B, sum exactly in a double
    rng = random.Random(400 + hi.bit_length())
    Ps = [1, 31, 32, 33, 64, 65, 96, 128, 150, 192, 200, 256, 260, 300, 320, 321, 384,
          400, 512, 600, 768, 800, 1000, 1088]
    cases = []
    for M in edge_moduli(lo, hi, rng)[:9]:
        bound = invariant(M, re, c)
        for x in (bound, -bound, 0, 1, -1, M // 2, -(M // 2), rng.randrange(-bound, bound + 1)):
            for P in Ps:
                cases.append((M, x, P, steps))
    lines = []
    for M, x, P, mode in cases:
        N, B = digit_layout(P)
        lines.append("D %d %d %d %d %d %d" % (M, x, P, B, N, mode))
    out = model(lines)
    for (M, x, P, mode), line in zip(cases, out):
        N, B = digit_layout(P)
        f = line.split()
        qs = [int(v) for v in f[:N]][::-1]          # q_0 (lowest) first
        neg, ok = int(f[N]), int(f[N + 1])
        assert ok == 1, (M, x, P)
        value = sum(q << (d * B) for d, q in enumerate(qs)) - neg
        assert value % 2 ** P == ((x % M) << P) // M % 2 ** P, (M, x, P)
        ne = -(-P // B)
        bt = P - (ne - 1) * B
        assert abs(qs[ne - 1]) <= 2 ** bt + 1, (M, x, P)
        assert all(abs(q) <= 2 ** (B - 1) + 2 ** (B - 6) + 1 for q in qs[:ne - 1]), (M, x, P)
        assert all(abs(q) <= 1 for q in qs[ne:]), (M, x, P)
        # a carried sum (below 2^B) plus CARRY_TERMS digits, minus the count of
        # negative remainders, plus the carry from below (at most 122)
        assert B <= 46 and N * B >= P
        assert 2 ** B + CARRY_TERMS * (2 ** B + 1) + CARRY_TERMS + 122 < 2 ** 53


def test_long_division_of_random_residues(model):
    # random moduli across the binary64 range, random residues and P
    rng = random.Random(1008)
    cases = []
    for _ in range(3000):
        M = rng.randrange(2 ** 29, 2 ** 51) | 1
        x = rng.randrange(-(M // 2), M // 2 + 1)
        P = rng.randrange(1, 1089)
        cases.append((M, x, P))
    out = model(["D %d %d %d %d %d 0" % (M, x, P, digit_layout(P)[1], digit_layout(P)[0])
                 for M, x, P in cases])
    for (M, x, P), line in zip(cases, out):
        N, B = digit_layout(P)
        f = line.split()
        qs = [int(v) for v in f[:N]][::-1]
        assert int(f[N + 1]) == 1
        value = sum(q << (d * B) for d, q in enumerate(qs)) - int(f[N])
        assert value % 2 ** P == ((x % M) << P) // M % 2 ** P, (M, x, P)
