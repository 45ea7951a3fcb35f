"""Pins of the oracle's certification and of its term count N.

Section 3.1 bounds the error of a truncated fixed-point BBP sum and warns
that a small error alone does not prove b bits: a run of 0s or of 1s right
below the last wanted bit can carry the true value across a bit boundary. The
oracle turns that into a two-sided test on the guard window (G >= B and
G + B <= 2^g, B = N + 2J units of 2^-P). These tests check

* the test itself against its definition, the interval of every real within
  B units of S, written with different arithmetic (a grid of half units, or
  the first multiple of 2^g above S - B), at every guard value of small
  windows and at the four edges G = B-1, B, 2^g-B, 2^g-B+1 of large ones;
* its soundness against pi: at every n up to 4000, with 10 to 15 guard bits,
  every certified window's bits equal Machin's (a different series for pi),
  and the scan does meet windows whose bits are wrong, all uncertified;
* N (every head index plus every tail index before the first zero
  truncation) against its definition, counted in Python integers;
* and that a mistake planted in a copy of the oracle's C (one side of the
  test dropped, the stop index counted, an index lost) fails these pins, and
  that a mistake planted in its arithmetic (a sign, a power, an exponent, a
  transposed operand, a shift, a reordered ladder) fails the arithmetic pins
  of the other test file, run here on the planted copy.
"""
import os
import random
from concurrent.futures import ThreadPoolExecutor
from fractions import Fraction

import pytest

import oracle
from conftest import machin_window

FORMULAS = [oracle.BBP, oracle.BELLARD]


# ---- certification against the interval definition -------------------------

def grid_certifies(S, P, w, B):
    """Every x with |x - S| < B (mod 2^P) has top w bits equal to S's, checked
    on the grid of half units: a boundary m 2^g strictly inside the interval
    has m 2^g and m 2^g - 1/2 both inside (the ends S -+ B are integers)."""
    g = P - w
    top = S >> g
    for y in range(2 * S - 2 * B + 1, 2 * S + 2 * B):   # x = y / 2
        if ((y % 2 ** (P + 1)) >> (g + 1)) != top:
            return False
    return True


def boundary_certifies(S, P, w, B):
    """The same definition for large B: the top bits of x change only at the
    multiples of 2^g (2^P is one of them), so the open interval (S - B, S + B)
    keeps them iff its first multiple of 2^g above S - B is at or past S + B."""
    g = P - w
    first = ((S - B) // 2 ** g + 1) * 2 ** g
    return first >= S + B


def check_certify_small(orc, P, w, Bs):
    for S in range(2 ** P):
        for B in Bs:
            assert orc.certify(S, P, w, B) == grid_certifies(S, P, w, B), (S, P, w, B)


def check_certify_edges(orc, rng, cases=60):
    for _ in range(cases):
        P = rng.choice([64, 96, 128, 320, 1088])
        w = rng.randrange(1, P - 20)
        g = P - w
        B = rng.randrange(2 * 7, min(2 ** 62, 2 ** (g - 2)))
        R = rng.randrange(2 ** w)
        for G in (B - 1, B, 2 ** g - B, 2 ** g - B + 1, rng.randrange(2 ** g)):
            S = (R << g) | G
            want = boundary_certifies(S, P, w, B)
            assert orc.certify(S, P, w, B) == want, (P, w, B, G)
        # the edges themselves: certified exactly at G = B and G = 2^g - B
        assert boundary_certifies((R << g) | B, P, w, B)
        assert boundary_certifies((R << g) | (2 ** g - B), P, w, B)
        assert not boundary_certifies((R << g) | (B - 1), P, w, B)
        assert not boundary_certifies((R << g) | (2 ** g - B + 1), P, w, B)


def test_certify_equals_interval_definition_at_every_guard_value():
    # every S of a 10-bit sum with 3 result bits (a 7-bit guard window), for
    # bounds below, at and past the half window
    check_certify_small(oracle, 10, 3, [0, 1, 2, 3, 5, 31, 63, 64, 65, 100, 127, 128])
    check_certify_small(oracle, 9, 9, [0, 1, 2])      # no guard bits at all


def test_certify_at_the_four_edges_of_large_windows():
    check_certify_edges(oracle, random.Random(31))


def test_grid_and_boundary_forms_agree():
    # the two written-out forms of the definition agree with each other
    rng = random.Random(5)
    for _ in range(3000):
        P = rng.randrange(2, 14)
        w = rng.randrange(1, P + 1)
        S = rng.randrange(2 ** P)
        B = rng.randrange(0, 2 ** (P - w) + 3)
        assert grid_certifies(S, P, w, B) == boundary_certifies(S, P, w, B)


# ---- soundness against pi ------------------------------------------------------

def scan_windows(orc, machin, nmax=4000, guards=(10, 11, 12, 13, 14, 15), w=16):
    jobs = [(f, n, g) for f in FORMULAS for n in range(1, nmax + 1) for g in guards]

    def one(job):
        f, n, g = job
        S, N, cert = orc.extract(f, n, w, w + g)
        return cert, S, N, machin_window(machin, n, w)

    with ThreadPoolExecutor(8) as ex:
        return jobs, list(ex.map(one, jobs))


def check_soundness(jobs, res, w=16):
    """Every window's flag is the interval definition at B = N + 2J (each of
    the N terms is truncated by less than one unit, each series' tail past its
    stop index adds less than 2^-P / (1 - 2^-step) <= 16/15 unit), and every
    certified window holds pi's bits."""
    certified = wrong = 0
    J = {f: len(oracle.series_table(f)[0]) for f in FORMULAS}
    for (f, n, g), (cert, S, N, ref) in zip(jobs, res):
        assert cert == boundary_certifies(S, w + g, w, N + 2 * J[f]), (f, n, g)
        if cert:
            certified += 1
            assert S >> g == ref, (f, n, g)
        elif S >> g != ref:
            wrong += 1
    return certified, wrong


def test_certified_windows_are_pis_bits(machin):
    jobs, res = scan_windows(oracle, machin)
    certified, wrong = check_soundness(jobs, res)
    # not vacuous: many windows certified, and some windows whose 16 bits are
    # not pi's (the runs-of-equal-bits case) were met and left uncertified
    assert certified > 10_000 and wrong > 100, (certified, wrong)


# ---- N against its definition ----------------------------------------------

def n_definition(formula, d, P, k0=0, k1=None):
    """Indices of [k0, k1) a sum adds, in Python integers: every head index
    (E = d + c - step k >= 0) and every tail index before the first one whose
    truncation floor(2^(P+E) / M) is 0 (the tail never grows again after it)."""
    rows, step, _ = oracle.series_table(formula)
    total = 0
    for sign, c, a, b in rows:
        K = (d + c) // step + 1 if d + c >= 0 else 0      # head: k < K
        hi = K if k1 is None else min(k1, K)
        total += max(0, hi - k0)
        k = max(k0, K)
        while (k1 is None or k < k1) and d + c - step * k + P >= 0 and \
                2 ** (d + c - step * k + P) >= a * k + b:
            total += 1
            k += 1
    return total


def test_n_equals_its_definition_for_whole_extractions():
    rng = random.Random(1008)
    cases = [(f, n, P) for f in FORMULAS for n in (1, 2, 3, 4, 5, 9, 10, 11, 100)
             for P in (1, 2, 7, 64)]
    for _ in range(320):
        f = rng.choice(FORMULAS)
        n = rng.randrange(1, 20_000)
        P = rng.choice([rng.randrange(1, 130), rng.randrange(1, 1089)])
        cases.append((f, n, P))
    for i, (f, n, P) in enumerate(cases):
        w = 1 + i % P
        S, N, cert = oracle.extract(f, n, w, P)
        Nd = n_definition(f, n - 1, P)
        assert N == Nd, (f, n, P)
        # the flag is the interval definition at B = N + 2J: each of the N terms
        # is truncated by less than one unit, and each series' tail past its
        # stop index adds less than 2^-P / (1 - 2^-step) <= 16/15 unit
        J = len(oracle.series_table(f)[0])
        assert cert == boundary_certifies(S, P, w, Nd + 2 * J), (f, n, w, P)


def test_n_equals_its_definition_for_slices_at_large_positions():
    rng = random.Random(3171)
    for _ in range(300):
        f = rng.choice(FORMULAS)
        rows, step, _ = oracle.series_table(f)
        j = rng.randrange(len(rows))
        d = rng.choice([rng.randrange(10 ** 6), rng.randrange(10 ** 12), 2 * 10 ** 15 - 4])
        P = rng.randrange(1, 1089)
        K = (d + rows[j][1]) // step + 1
        # ranges around the head/tail boundary and the stop index
        k0 = max(0, K - rng.randrange(0, 300))
        k1 = k0 + rng.randrange(0, 400)
        S, N = oracle.sum_slice(f, j, d, k0, k1, P)
        one = n_definition_series(f, j, d, P, k0, k1)
        assert N == one, (f, j, d, P, k0, k1)


def n_definition_series(formula, j, d, P, k0, k1):
    rows, step, _ = oracle.series_table(formula)
    sign, c, a, b = rows[j]
    count = 0
    for k in range(k0, k1):
        E = d + c - step * k
        if E >= 0:
            count += 1
        elif E + P >= 0 and 2 ** (E + P) >= a * k + b:
            count += 1
        else:
            break
    return count


# ---- planted mistakes fail the pins -------------------------------------------

# Each mistake is a textual change of the oracle's C that a careless edit could
# make; the test builds that copy on the CPU and checks that some pin above
# rejects it.
MISTAKES = {
    "certify without the lower edge (G >= B)": ("return ge && le;", "return le;"),
    "certify without the upper edge (G + B <= 2^g)": ("return ge && le;", "return ge;"),
    "the stop index counted in N": (
        "if (E < 0 && is_zero(t, nw)) break;",
        "if (E < 0 && is_zero(t, nw)) { jb->nterms++; break; }"),
    "zero head terms (2^E mod 1) left out of N": (
        "    jb->nterms++;", "    if (!is_zero(t, nw)) jb->nterms++;"),
    "an error bound of N + J instead of N + 2J": (
        "total + 2u * (uint64_t)J", "total + (uint64_t)J"),
}


def planted(tmp_path, old, new):
    here = os.path.dirname(oracle.__file__)
    src = open(os.path.join(here, "pio.c")).read()
    assert src.count(old) == 1, old
    (tmp_path / "pio.h").write_text(open(os.path.join(here, "pio.h")).read())
    path = tmp_path / "pio_planted.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / "libpio_planted.so")
    oracle.compile_source(str(path), lib)
    return oracle.Oracle(lib)


def pins_pass(orc, machin):
    """The pins above, on another copy of the oracle; False at the first
    failure."""
    try:
        check_certify_small(orc, 10, 3, [0, 1, 2, 3, 5, 31, 63, 64, 65, 100, 127, 128])
        check_certify_edges(orc, random.Random(31), cases=20)
        jobs, res = scan_windows(orc, machin, nmax=1500, guards=(10, 12, 14))
        certified, wrong = check_soundness(jobs, res)
        assert certified > 1000 and wrong > 10
        rng = random.Random(1008)
        for i in range(120):
            f = rng.choice(FORMULAS)
            n = rng.randrange(1, 20_000)
            P = rng.randrange(1, 1089)
            w = 1 + i % P
            S, N, cert = orc.extract(f, n, w, P)
            Nd = n_definition(f, n - 1, P)
            assert N == Nd
            J = len(oracle.series_table(f)[0])
            assert cert == boundary_certifies(S, P, w, Nd + 2 * J)
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_planted_mistake_fails_a_pin(name, tmp_path, machin):
    old, new = MISTAKES[name]
    assert not pins_pass(planted(tmp_path, old, new), machin), name


def test_unchanged_copy_passes_the_same_pins(tmp_path, machin):
    # the copy-and-build route itself changes nothing
    assert pins_pass(planted(tmp_path, "return ge && le;", "return ge && le;"), machin)


# ---- planted arithmetic mistakes fail the arithmetic pins -------------------

ARITH_MISTAKES = {
    "a wrong sign in one of Bellard's series": ("{-1, -4, 10, 5}", "{+1, -4, 10, 5}"),
    "a BBP denominator not halved (wrong power of two)": ("{-1, -1, 2, 1}", "{-1, 0, 2, 1}"),
    "the alternating sign dropped": (
        "int neg = (jb->sr.sign < 0) ^ (jb->alt < 0 && (k & 1u));",
        "int neg = (jb->sr.sign < 0);"),
    "a term's exponent off by one": (
        "  int64_t E = (int64_t)d + sr->c - (int64_t)step * (int64_t)k;\n  uint64_t M",
        "  int64_t E = (int64_t)d + sr->c - (int64_t)step * (int64_t)k + 1;\n  uint64_t M"),
    "the modulus's operands transposed (b k + a)": (
        "uint64_t M = sr->a * k + sr->b;", "uint64_t M = sr->b * k + sr->a;"),
    "a tail term's precision off by one": (
        "int64_t bits = (int64_t)P + E;", "int64_t bits = (int64_t)P + E - 1;"),
    "the quotient's final shift off by one": (
        "uint32_t s = 32u * nd - bits;", "uint32_t s = 32u * nd - bits + 1u;"),
    "the ladder squares before it multiplies": (
        "    if (e & 1u) result = (uint64_t)((u128)result * base % m);\n"
        "    base = (uint64_t)((u128)base * base % m);",
        "    base = (uint64_t)((u128)base * base % m);\n"
        "    if (e & 1u) result = (uint64_t)((u128)result * base % m);"),
}


def printed_formula(formula, kmax):
    """eq (1.1) or (1.2) as printed, summed to kmax in exact rationals."""
    F = Fraction
    tot = F(0)
    for k in range(kmax):
        if formula == oracle.BBP:
            tot += F(1, 16 ** k) * (F(4, 8 * k + 1) - F(2, 8 * k + 4) - F(1, 8 * k + 5)
                                    - F(1, 8 * k + 6))
        else:
            tot += F((-1) ** k, 2 ** (10 * k)) * (
                F(4, 10 * k + 1) - F(1, 10 * k + 3) - F(1, 16 * (10 * k + 5))
                - F(1, 16 * (10 * k + 7)) + F(1, 64 * (10 * k + 9))
                - F(1, 2 * (4 * k + 1)) - F(1, 64 * (4 * k + 3)))
    return tot


# The series of the printed formulas in the form sign 2^c / (a k + b), written
# out here (not read from the oracle) and pinned to the printed formulas below.
WRITTEN = {
    oracle.BBP: (4, +1, [(+1, 2, 8, 1), (-1, -1, 2, 1), (-1, 0, 8, 5), (-1, -1, 4, 3)]),
    oracle.BELLARD: (10, -1, [(+1, 2, 10, 1), (-1, 0, 10, 3), (-1, -4, 10, 5), (-1, -4, 10, 7),
                              (+1, -6, 10, 9), (-1, -1, 4, 1), (-1, -6, 4, 3)]),
}


def exact_term_printed(formula, j, d, k, P):
    """floor(2^P frac(2^E / M)) from exact rationals, with the series of
    WRITTEN."""
    step, _, rows = WRITTEN[formula]
    _, c, a, b = rows[j]
    E, M = d + c - step * k, a * k + b
    x = Fraction(2 ** E, M) if E >= 0 else Fraction(1, 2 ** (-E) * M)
    v = (x - x.numerator // x.denominator) * 2 ** P
    return v.numerator // v.denominator


def arith_pins_pass(orc, machin):
    """The arithmetic pins of the other oracle test file, on another copy of
    the oracle: the tables sum to the printed formulas, the modular power
    equals Python's, terms equal exact rationals, and certified windows hold
    Machin's bits. False at the first failure."""
    try:
        for f, kmax in ((oracle.BBP, 40), (oracle.BELLARD, 20)):
            rows, step, alt = orc.series_table(f)
            tot = sum(sign * alt ** k * Fraction(2) ** (c - step * k) / (a * k + b)
                      for k in range(kmax) for sign, c, a, b in rows)
            assert tot == printed_formula(f, kmax)
        rng = random.Random(77)
        for _ in range(300):
            m = rng.randrange(1, 2 ** rng.randrange(1, 63))
            e = rng.randrange(0, 2 ** 62)
            assert orc.pow2mod(e, m) == pow(2, e, m)
        for f in FORMULAS:
            J = 4 if f == oracle.BBP else 7
            step = 4 if f == oracle.BBP else 10
            for _ in range(200):
                d = rng.randrange(0, 200)
                j = rng.randrange(J)
                k = rng.randrange(0, d // step + 30)
                P = rng.choice([1, 7, 31, 32, 33, 63, 64, 65, 96, 128, 200])
                assert orc.term(f, j, d, k, P) == exact_term_printed(f, j, d, k, P)
        certified = 0
        for f in FORMULAS:
            for n in range(1, 301):
                S, N, cert = orc.extract(f, n, 16, 48)
                if cert:
                    certified += 1
                    assert S >> 32 == machin_window(machin, n, 16)
        assert certified > 550
    except AssertionError:
        return False
    return True


def test_written_out_series_are_the_printed_formulas():
    for f, kmax in ((oracle.BBP, 30), (oracle.BELLARD, 15)):
        step, alt, rows = WRITTEN[f]
        tot = sum(sign * alt ** k * Fraction(2) ** (c - step * k) / (a * k + b)
                  for k in range(kmax) for sign, c, a, b in rows)
        assert tot == printed_formula(f, kmax)


@pytest.mark.parametrize("name", sorted(ARITH_MISTAKES))
def test_planted_arithmetic_mistake_fails_a_pin(name, tmp_path, machin):
    old, new = ARITH_MISTAKES[name]
    assert not arith_pins_pass(planted(tmp_path, old, new), machin), name


def test_unchanged_copy_passes_the_arithmetic_pins(tmp_path, machin):
    assert arith_pins_pass(planted(tmp_path, "return ge && le;", "return ge && le;"), machin)
