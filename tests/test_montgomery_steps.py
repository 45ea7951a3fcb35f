"""The head kernel's integer Montgomery steps (section 4.2 names Montgomery's
method for the modular exponentiation), modelled on the CPU word by word.

Each model below repeats one device routine of the integer classes with the
register widths of the kernel: every 32-bit product or sum is taken modulo
2^32 where the kernel's register is 32 bits, and every 64-bit multiply-add is
asserted to stay below 2^64 where the kernel drops the carry. The models are
then checked against Python's exact arithmetic (pow, //, modular inverse) at
the edges the kernel's comments bound:

* the R = 2^62 squaring on two 31-bit digits (moduli from 2^31 to 2^54 in
  integer mode, from 2^51 by default): x < 8M in, REDC below 2.26M, below
  4.52M after the doubling; the first squaring of a lane run from its start
  value g 2^v with (g 2^v)^2 < 2^60 M and g 2^v < 2^56;
* the lazy R = 2^32 squaring (moduli below 2^30), plain and with a window
  digit d (2^(d+2) M < 2^32), inputs and outputs below 2M, and the reduced
  form of 2^29 <= M < 2^31;
* -M^-1 mod 2^32 by Newton steps from a 5-bit seed, the quotients
  floor(2^62 / M) and floor(2^32 / M), the Montgomery one 2^32 mod M, and
  whole ladders of each class against pow(2, X, M).
"""
import random

import pytest

M32 = 2 ** 32 - 1
M31 = 2 ** 31 - 1
TWO64 = 2 ** 64


def mad64(a, b, c):
    """v_mad_u64_u32 as the kernel uses it: a b + c with a, b 32-bit and c
    64-bit, the carry out dropped; the kernel's bounds say there is none."""
    assert 0 <= a <= M32 and 0 <= b <= M32 and 0 <= c < TWO64
    v = a * b + c
    assert v < TWO64, "64-bit multiply-add overflows"
    return v


def neg_inv32(m):
    """-M^-1 mod 2^32: (3M) xor 2 is right to 5 bits, and each step
    x <- x (2 - M x) doubles the correct bits (5, 10, 20, 40)."""
    x = ((3 * m) & M32) ^ 2
    for _ in range(3):
        x = (x * ((2 - m * x) & M32)) & M32
    return (-x) & M32


def sqr_redc62(d0, d1, b, m0, m1, p):
    """x <- 2^b REDC(x^2) with R = 2^62 on 31-bit digits x = d0 + d1 2^31."""
    c0 = d0 * d0
    u0 = ((c0 & M32) * p) & M32
    c0 = mad64(u0, m0, c0)
    c1 = mad64(d0, (d1 << 1) & M32, c0 >> 31)
    c1 = mad64(u0, m1, c1)
    u1 = ((c1 & M32) * p) & M32
    c1 = mad64(u1, m0, c1)
    c2 = mad64(d1, d1, c1 >> 31)
    c2 = mad64(u1, m1, c2)
    c2 = (c2 << b) & (TWO64 - 1)
    return c2 & M31, (c2 >> 31) & M32


def redc62_step(x, b, M):
    """The squaring on x (any integer the digits hold), returning the new x."""
    mp32 = neg_inv32(M & M32)
    d0, d1 = x & M31, x >> 31
    assert d1 <= M32
    e0, e1 = sqr_redc62(d0, d1, b, M & M31, M >> 31, mp32 & M31)
    return e0 + (e1 << 31)


def sqr_redc32_plain(x, M, mp):
    T = x * x
    assert T < TWO64
    q = ((T & M32) * mp) & M32
    v = T + q * M
    assert v < TWO64
    return (v >> 32) & M32


def sqr_redc32_digit(x, d, M, mp):
    xs = (x << d)
    assert xs <= M32, "x 2^d leaves its 32-bit register"
    T = x * xs
    q = ((T & M32) * mp) & M32
    v = T + q * M
    assert v < TWO64
    return (v >> 32) & M32


def div_2_62(M):
    """floor(2^62 / M) for 2^31 <= M < 2^54 by restoring division; bit s is
    tried only while M 2^s stays below 2^63."""
    room = 63 - M.bit_length()
    r, q = 1 << 62, 0
    for s in range(31, -1, -1):
        if s <= room:
            ms = M << s
            if r >= ms:
                r -= ms
                q |= 1 << s
    return q


def div_2_32(M):
    r, q = 1 << 32, 0
    for s in range(10, -1, -1):
        if r >= (M << s):
            r -= M << s
            q |= 1 << s
    return q


def mont_one32(M):
    bl = M.bit_length()
    c = (1 << bl) - M
    for _ in range(bl, 32):
        c = (c << 1) & M32
        c = min(c, (c - M) & M32)
    return c


def moduli(lo, hi, rng, count=40):
    ms = [lo | 1, (lo + 2) | 1, hi - 1, hi - 3, hi - 21]
    ms += [rng.randrange(lo, hi) | 1 for _ in range(count)]
    return [m for m in ms if lo <= m < hi]


# ---- the R = 2^62 class ----------------------------------------------------------

def test_redc62_edges_against_pow():
    rng = random.Random(62)
    for M in moduli(2 ** 31, 2 ** 54, rng) + [2 ** 31 + 1, 2 ** 54 - 1, 2 ** 51 + 1, 2 ** 36 - 1]:
        R_inv = pow(2 ** 62, -1, M)
        for x in (0, 1, 2, M - 1, M, M + 1, 2 * M - 1, 4 * M + 7, 8 * M - 1,
                  rng.randrange(8 * M)):
            for b in (0, 1):
                y = redc62_step(x, b, M)
                assert (y - x * x * 2 ** b * R_inv) % M == 0, (M, x, b)
                # REDC below 2.26 M, below 4.52 M after the doubling
                assert y < (2.26 if b == 0 else 4.52) * M, (M, x, b)
                assert y < 8 * M


def test_redc62_first_squaring_from_run_start_values():
    # a lane run starts from g = 2^62 - qM with q = floor(2^62 / M_last),
    # shifted left by v top exponent bits; the planner keeps
    # (g 2^v)^2 < 2^60 M and g 2^v < 2^56, and the first squaring must then
    # land below 8M
    rng = random.Random(63)
    for M in moduli(2 ** 31, 2 ** 54, rng, 200):
        R_inv = pow(2 ** 62, -1, M)
        lim = min(2 ** 56, int((2 ** 60 * M) ** 0.5))
        for x in (lim - 1, lim // 2, rng.randrange(lim)):
            for b in (0, 1):
                y = redc62_step(x, b, M)
                assert (y - x * x * 2 ** b * R_inv) % M == 0
                assert y < 8 * M, (M, x, b)


def test_quotient_2_62_and_start_value():
    rng = random.Random(64)
    for M in moduli(2 ** 31, 2 ** 54, rng, 300):
        q = div_2_62(M)
        assert q == 2 ** 62 // M
        g = 2 ** 62 - q * M
        assert 0 <= g < M and g % M == 2 ** 62 % M


def ladder62(X, M, pre=0):
    """The class-62 ladder in Montgomery form (R = 2^62): the start value
    2^62 - qM == R (mod M) is the form of 1, shifted left by the top `pre`
    bits v of X it is the form of 2^v, and each remaining bit of X squares
    with that bit as the doubling; the result, brought below M, is the form
    R 2^X of 2^X."""
    nb0 = X.bit_length()
    tb = min(pre, nb0)
    nb = nb0 - tb
    v = (X >> nb) & ((1 << tb) - 1)
    x = (2 ** 62 - div_2_62(M) * M) << v
    for j in range(nb - 1, -1, -1):
        x = redc62_step(x, (X >> j) & 1, M)
        assert x < 8 * M              # the input bound of every later squaring
    for s in (4, 2, 1):               # the kernel's reduction from below 8M
        if x >= s * M:
            x -= s * M
    return x


def test_ladder62_equals_pow():
    # with X = E + 64L - 62 the form R 2^X is 2^(E + 64L) mod M, the s the
    # Hensel division needs
    rng = random.Random(65)
    for M in moduli(2 ** 31, 2 ** 54, rng, 30):
        for _ in range(6):
            E = rng.randrange(0, 2 ** 52)
            L = rng.choice([1, 2, 5, 17])
            for pre in (0, 1, 2, 3):
                # the planner's rule for the start bits: the largest start
                # value g 2^v, v < 2^pre, has (g 2^v)^2 < 2^60 M and is below 2^56
                top = (2 ** 62 - div_2_62(M) * M) << ((1 << pre) - 1)
                if top * top >= 2 ** 60 * M or top >= 2 ** 56:
                    continue
                x = ladder62(E + 64 * L - 62, M, pre)
                assert x == pow(2, E + 64 * L, M), (M, E, L, pre)


# ---- the R = 2^32 classes --------------------------------------------------------

def test_redc32_plain_and_digit_edges():
    rng = random.Random(32)
    cases = []
    # (lowest modulus, first modulus past the class, window bits)
    for lo, hi, W in ((3, 2 ** 22, 3), (2 ** 22, 2 ** 27, 2), (2 ** 27, 2 ** 29, 1),
                      (2 ** 29, 2 ** 30, 1)):
        for M in moduli(lo, hi, rng, 30):
            cases.append((M, W))
    for M, W in cases:
        mp = neg_inv32(M)
        assert (M * mp) % 2 ** 32 == 2 ** 32 - 1
        R_inv = pow(2 ** 32, -1, M)
        for x in (0, 1, M - 1, M, 2 * M - 1, rng.randrange(2 * M)):
            y = sqr_redc32_plain(x, M, mp)
            assert (y - x * x * R_inv) % M == 0 and y < 2 * M, (M, x)
            for d in range(1 << W):
                if 2 ** (d + 2) * M >= 2 ** 32:
                    continue        # the kernel never pairs this digit with this modulus
                y = sqr_redc32_digit(x, d, M, mp)
                assert (y - x * x * 2 ** d * R_inv) % M == 0 and y < 2 * M, (M, x, d)


def test_redc32_window_digits_cover_their_classes():
    # every digit a class uses satisfies 2^(d+2) M < 2^32 at its largest modulus
    for hi, W in ((2 ** 22, 3), (2 ** 23, 3), (2 ** 27, 2), (2 ** 29, 1)):
        assert 2 ** ((1 << W) - 1 + 2) * (hi - 1) < 2 ** 32


def test_reduced_class_from_2_29():
    # 2^29 <= M < 2^31 (integer mode): residues reduced below M after every
    # step, so x (x << b) < 2 M^2 and REDC stays below 2M
    rng = random.Random(31)
    for M in moduli(2 ** 29, 2 ** 31, rng, 60):
        mp = neg_inv32(M)
        R_inv = pow(2 ** 32, -1, M)
        for x in (0, 1, M - 1, rng.randrange(M)):
            for b in (0, 1):
                y = sqr_redc32_digit(x, b, M, mp)
                assert y < 2 * M and (y - x * x * 2 ** b * R_inv) % M == 0
                y = min(y, (y - M) & M32)
                assert y < M


def test_quotient_2_32_montgomery_one_and_inverse():
    rng = random.Random(33)
    for M in moduli(2 ** 22, 2 ** 31, rng, 300):
        assert div_2_32(M) == 2 ** 32 // M
    # the run-quotient start: a lane's run of moduli M, M + 2a, ... shares
    # q = floor(2^32 / M_last), and the planner caps the run at
    # floor(Mmin^2 / 2^32 / 2a) so that g = 2^32 - qM stays below 2M
    for a in (2, 4, 8, 10):
        for Mmin in moduli(2 ** 22, 2 ** 31, rng, 60):
            run = max(1, (Mmin * Mmin >> 32) // (2 * a))
            Mlast = Mmin + 2 * a * (run - 1)
            q = div_2_32(Mlast)
            for M in (Mmin, Mmin + 2 * a * (run // 2), Mlast):
                g = (-(q * M)) & M32
                assert g % M == 2 ** 32 % M and g < 2 * M, (a, Mmin, run, M)
    for M in moduli(3, 2 ** 31, rng, 300) + [3, 5, 7, 2 ** 31 - 1]:
        assert mont_one32(M) == 2 ** 32 % M
        assert (neg_inv32(M) * M + 1) % 2 ** 32 == 0
    for m in range(1, 1 << 12, 2):            # every odd low part
        assert (neg_inv32(m) * m + 1) % 2 ** 32 == 0


def ladder32(X, M, W):
    """The class-32 ladder: a short leading window of bitlen mod W bits, then
    whole W-bit windows, each W-1 plain squarings and one with its digit,
    from the Montgomery one 2^32 mod M; ends reduced below M."""
    mp = neg_inv32(M)
    nb = X.bit_length()
    lead = nb % W
    top = nb - lead
    x = mont_one32(M)
    if lead:
        for _ in range(lead - 1):
            x = sqr_redc32_plain(x, M, mp)
        x = sqr_redc32_digit(x, (X >> top) & ((1 << lead) - 1), M, mp)
    for p in range(top - W, -1, -W):
        for _ in range(W - 1):
            x = sqr_redc32_plain(x, M, mp)
        x = sqr_redc32_digit(x, (X >> p) & ((1 << W) - 1), M, mp)
    return min(x, (x - M) & M32)


@pytest.mark.parametrize("lo,hi,W", [(3, 2 ** 22, 3), (2 ** 22, 2 ** 27, 2),
                                     (2 ** 27, 2 ** 29, 1)])
def test_ladder32_equals_pow(lo, hi, W):
    rng = random.Random(hi)
    for M in moduli(lo, hi, rng, 25):
        for _ in range(8):
            E = rng.randrange(0, 2 ** 40)
            L = rng.choice([1, 2, 5, 17])
            X = E + 64 * L - 32
            x = ladder32(X, M, W)
            assert x == pow(2, E + 64 * L, M), (M, E, L, W)
