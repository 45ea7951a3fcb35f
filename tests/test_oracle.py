"""Pins of the oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the paper's
printed bits, Machin's formula (a different series for pi), exact rational
arithmetic on tiny inputs, Python's built-in modular power, the division
identity, and agreement between two different BBP-type formulas.
"""
import random
from concurrent.futures import ThreadPoolExecutor
from fractions import Fraction

import pytest

import oracle
from conftest import hex_bits, machin_window, read_golden

FORMULAS = [oracle.BBP, oracle.BELLARD]


def exact_term(formula, j, d, k, P):
    """floor(2^P * frac(2^E / M)) from exact rationals (tiny inputs only)."""
    rows, step, _ = oracle.series_table(formula)
    sign, c, a, b = rows[j]
    E = d + c - step * k
    M = a * k + b
    x = Fraction(2 ** E, M) if E >= 0 else Fraction(1, 2 ** (-E) * M)
    frac = x - (x.numerator // x.denominator)
    v = frac * 2 ** P
    return v.numerator // v.denominator


@pytest.mark.parametrize("formula", FORMULAS)
def test_worked_example(formula):
    # footnote to the abstract: bits 9..16 are 0x3F; pi = 11.0010 0100 0011 1111...
    for n, nbits, h in read_golden("worked_example.txt"):
        n, nbits = int(n), int(nbits)
        S, N, cert = oracle.extract(formula, n, nbits, nbits + 64)
        assert cert
        assert S >> 64 == int(h, 16)


def test_formulas_as_written_sum_to_pi(machin):
    # Evaluate (1.1) and (1.2) exactly as printed, with rationals, and compare
    # with Machin; this pins the series tables (signs, powers, denominators).
    nbits = 256
    bbp = Fraction(0)
    bel = Fraction(0)
    for k in range(80):
        bbp += Fraction(1, 16 ** k) * (Fraction(4, 8 * k + 1) - Fraction(2, 8 * k + 4)
                                       - Fraction(1, 8 * k + 5) - Fraction(1, 8 * k + 6))
    for k in range(40):
        bel += Fraction((-1) ** k, 2 ** (10 * k)) * (
            Fraction(4, 10 * k + 1) - Fraction(1, 10 * k + 3) - Fraction(1, 16 * (10 * k + 5))
            - Fraction(1, 16 * (10 * k + 7)) + Fraction(1, 64 * (10 * k + 9))
            - Fraction(1, 2 * (4 * k + 1)) - Fraction(1, 64 * (4 * k + 3)))
    ref = machin_window(machin, 1, nbits)
    for val in (bbp, bel):
        frac = val - 3
        assert (frac * 2 ** nbits).__floor__() == ref
    # and the tables reproduce the same sums term by term
    for formula, val in ((oracle.BBP, bbp), (oracle.BELLARD, bel)):
        rows, step, alt = oracle.series_table(formula)
        tot = Fraction(0)
        for k in range(80 if formula == oracle.BBP else 40):
            for sign, c, a, b in rows:
                tot += sign * alt ** k * Fraction(2) ** (c - step * k) / (a * k + b)
        assert tot == val


def test_pow2mod_against_builtin():
    rng = random.Random(1008)
    cases = [(0, 1), (5, 1), (0, 7), (1, 3), (63, 2 ** 61 - 1), (10 ** 15, 2 ** 50 + 1)]
    for _ in range(2000):
        m = rng.randrange(1, 2 ** rng.randrange(1, 63))
        cases.append((rng.randrange(0, 2 ** 62), m))
    for e, m in cases:
        assert oracle.pow2mod(e, m) == pow(2, e, m)


@pytest.mark.parametrize("formula", FORMULAS)
def test_term_brute_force(formula):
    rng = random.Random(3171 + formula)
    rows, step, _ = oracle.series_table(formula)
    for _ in range(600):
        d = rng.randrange(0, 200)
        j = rng.randrange(len(rows))
        k = rng.randrange(0, d // step + 30)
        P = rng.choice([1, 7, 31, 32, 33, 63, 64, 65, 96, 128, 200])
        assert oracle.term(formula, j, d, k, P) == exact_term(formula, j, d, k, P)


def test_division_identity():
    # r * 2^P = t*M + s with 0 <= s < M, for the head terms of real workloads
    rng = random.Random(7)
    rows, step, _ = oracle.series_table(oracle.BELLARD)
    for _ in range(500):
        d = rng.choice([10 ** 6, 10 ** 10, 10 ** 12, 2 * 10 ** 15 - 4])
        j = rng.randrange(7)
        sign, c, a, b = rows[j]
        k = rng.randrange(0, (d + c) // step + 1)
        P = rng.choice([64, 96, 128, 192, 320, 1024])
        E, M = d + c - step * k, a * k + b
        t = oracle.term(oracle.BELLARD, j, d, k, P)
        r = pow(2, E, M)
        s = r * 2 ** P - t * M
        assert 0 <= s < M and 0 <= t < 2 ** P


def _check_window(args):
    formula, n, w, mach = args
    S, N, cert = oracle.extract(formula, n, w, w + 64)
    return cert, S >> 64, machin_window(mach, n, w)


def test_machin_every_position_below_2000(machin):
    jobs = [(f, n, 32, machin) for f in FORMULAS for n in range(1, 2001)]
    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(_check_window, jobs))
    for (f, n, _, _), (cert, got, ref) in zip(jobs, res):
        assert cert, (f, n)
        assert got == ref, (f, n)


def test_machin_sampled_to_1e5(machin):
    rng = random.Random(1008)
    ns = sorted(rng.randrange(2000, 100_000) for _ in range(40))
    jobs = [(f, n, w, machin) for f in FORMULAS for n in ns for w in (64, 256)]
    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(_check_window, jobs))
    for job, (cert, got, ref) in zip(jobs, res):
        assert cert, job[:3]
        assert got == ref, job[:3]


def test_bbp_and_bellard_agree_and_n_minus_4_overlaps():
    # Cross-formula agreement, and the paper's n / n-4 practice (section 3.1):
    # bits certified by both runs must coincide on their overlap.
    rng = random.Random(42)
    for _ in range(20):
        n = rng.randrange(5, 300_000)
        w = 64
        a = oracle.extract(oracle.BELLARD, n, w, w + 64, 8)
        b = oracle.extract(oracle.BBP, n, w, w + 64, 8)
        c = oracle.extract(oracle.BELLARD, n - 4, w, w + 64, 8)
        assert a[2] and b[2] and c[2]
        assert a[0] >> 64 == b[0] >> 64
        assert (c[0] >> 64) & ((1 << (w - 4)) - 1) == (a[0] >> 64) >> 4


def test_slice_additivity_and_partition_invariance():
    rng = random.Random(99)
    for formula in FORMULAS:
        rows, step, _ = oracle.series_table(formula)
        for _ in range(10):
            d = rng.randrange(10, 20_000)
            P = rng.choice([64, 96, 320])
            S, N, _ = oracle.extract(formula, d + 1, 32, P)
            tot = 0
            cnt = 0
            for j in range(len(rows)):
                kend = (d + 2) // step + P + 10          # past every nonzero tail term
                cuts = sorted(rng.sample(range(1, kend), 5))
                edges = [0] + cuts + [kend]
                for lo, hi in zip(edges, edges[1:]):
                    part, c = oracle.sum_slice(formula, j, d, lo, hi, P, rng.choice([1, 3]))
                    tot += part
                    cnt += c
            assert tot % 2 ** P == S
            assert cnt == N


def test_uncertain_when_guard_window_is_too_small():
    # With only 4 guard bits the error bound (N + 2J units) cannot fit in the
    # guard window, so nothing is certified, whatever the bits are.
    S, N, cert = oracle.extract(oracle.BELLARD, 1000, 32, 36)
    assert not cert and N + 14 > 16


def test_printed_rows_are_consistent():
    # section 3.1's true bits at 10^15+53 are row m=15 of Table 2.2 from offset 52
    (n, nb, true_hex, _), = read_golden("float64_demo.txt")
    rows = {int(r[0]): r for r in read_golden("table_2_2.txt")}
    m15 = rows[15]
    assert int(n) - int(m15[1]) == 52
    bits15 = hex_bits(m15[3], int(m15[2]))
    window = (bits15 >> (int(m15[2]) - 52 - 52)) & ((1 << 52) - 1)
    assert window == int(true_hex, 16)


@pytest.mark.slow
def test_table_2_2_row_m9():
    # 10^9 + 1: about 7*10^8 terms, ~1 min on 8 threads
    row = [r for r in read_golden("table_2_2.txt") if r[0] == "9"][0]
    n = int(row[1])
    S, N, cert = oracle.extract(oracle.BELLARD, n, 256, 320, 8)
    assert cert
    assert S >> 64 == hex_bits(row[3], 256)


@pytest.mark.slow
@pytest.mark.skipif(not __import__("os").environ.get("PIBBP_LONG"),
                    reason="7*10^9 terms, ~10 min on 8 threads; set PIBBP_LONG=1 to run")
def test_table_2_2_row_m10():
    row = [r for r in read_golden("table_2_2.txt") if r[0] == "10"][0]
    S, N, cert = oracle.extract(oracle.BELLARD, int(row[1]), 256, 320, 8)
    assert cert
    assert S >> 64 == hex_bits(row[3], 256)
