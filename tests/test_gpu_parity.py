"""Parity of the HIP library with the oracle, through the C ABI.

Every comparison is of the full P-bit sum S (bit-exact), plus N and the
certification flag where the call reports them. Sizes: small cases that span
many workgroup chunks and ragged ends, both modulus classes and their
boundary, every limb class, the degenerate positions, and sampled slices of
the full-size workloads.
"""
import random

import pytest

import oracle
import paper_1008_3171_amd as pb
from conftest import hex_bits, read_golden

pytestmark = pytest.mark.gpu

FORMULAS = [pb.BBP, pb.BELLARD]


def gpu_extract(formula, n, w, P):
    out, st = pb.extract(formula, n, w, P)
    S = pb.to_int(out, P)
    code, N = pb.status_of(st)
    return S, N, code == pb.PI_OK


def gpu_slice(formula, j, n, k0, k1, P):
    return pb.to_int(pb.sum_slice(pb.term_id(formula, j), n, k0, k1, P), P)


@pytest.mark.parametrize("formula", FORMULAS)
def test_worked_example(formula):
    for n, nbits, h in read_golden("worked_example.txt"):
        n, nbits = int(n), int(nbits)
        S, N, cert = gpu_extract(formula, n, nbits, nbits + 64)
        assert (S, N, cert) == oracle.extract(formula, n, nbits, nbits + 64)
        assert cert and S >> 64 == int(h, 16)


def test_small_positions_every_limb_class():
    rng = random.Random(1008)
    cases = [(f, n, w, P) for f in FORMULAS for n in (1, 2, 3, 5, 6, 7, 10, 11)
             for (w, P) in ((1, 1), (8, 64), (8, 65), (32, 96))]
    for _ in range(60):
        f = rng.choice(FORMULAS)
        n = rng.randrange(1, 300_000)
        P = rng.choice([64, 96, 128, 192, 256, 320, 384, 448, 512, 640, 768, 1024, 1088,
                        rng.randrange(1, 1089)])
        w = rng.randrange(1, P + 1)
        cases.append((f, n, w, P))
    for f, n, w, P in cases:
        got = gpu_extract(f, n, w, P)
        want = oracle.extract(f, n, w, P, 8)
        assert got == want, (f, n, w, P)


def test_bellard_n1e6_64_bits_P96():
    # 700,001 head terms, moduli < 2^20, 64 result bits + 32 guard bits
    got = gpu_extract(pb.BELLARD, 10 ** 6, 64, 96)
    want = oracle.extract(oracle.BELLARD, 10 ** 6, 64, 96, 8)
    assert got == want
    assert want[2]


@pytest.mark.parametrize("cut", [22, 27, 29, 31, 33, 42, 46, 48, 51])
def test_slices_across_every_modulus_class_boundary(cut):
    # the head kernel switches arithmetic where the modulus reaches 2^22, 2^27
    # and 2^29 (32-bit Montgomery with three-, two- and one-bit windows),
    # 2^33, 2^42, 2^48 and 2^51 (binary64 windows of four, three and two bits,
    # five bits with the digit applied after the squarings, then R = 2^62);
    # 2^31 and 2^46 are former cuts, kept as inner points:
    # ranges straddling each cut for every series, with exponents just past
    # the cut and near 2^61 (both halves of a 64-bit exponent)
    rng = random.Random(5 + cut)
    for f in FORMULAS:
        rows, step, _ = oracle.series_table(f)
        for j, (s, c, a, b) in enumerate(rows):
            ks = (2 ** cut - b + a - 1) // a
            for n in (step * ks + 10 ** 6, 2 ** 61 + rng.randrange(10 ** 6)):
                k0 = ks - rng.randrange(0, 3000)
                k1 = ks + rng.randrange(1, 3000)
                P = rng.choice([96, 320, 1088])
                assert gpu_slice(f, j, n, k0, k1, P) == \
                    oracle.sum_slice(f, j, n - 1, k0, k1, P, 8)[0], (f, j, n, k0, k1, P)


def test_binary64_division_every_limb_class_and_ragged_widths():
    # the binary64 classes (2^29 <= M < 2^51) divide each residue out in
    # digits of up to 46 bits, the top digit taking what is left of P and the
    # digits above it none: P at both ends of every limb class and in between
    rng = random.Random(64)
    Ps = [1, 31, 33, 64, 65, 100, 128, 150, 192, 200, 256, 260, 300, 320, 321, 384, 400,
          511, 512, 600, 768, 800, 1000, 1088]
    for i, P in enumerate(Ps):
        f = FORMULAS[i % 2]
        rows, step, _ = oracle.series_table(f)
        j = rng.randrange(len(rows))
        s, c, a, b = rows[j]
        for e in (30, 37, 45, 50):
            ks = (2 ** e - b) // a
            n = step * ks + rng.randrange(10 ** 6, 10 ** 9)
            k0 = ks + rng.randrange(0, 1000)
            k1 = k0 + rng.randrange(1, 5000)
            assert gpu_slice(f, j, n, k0, k1, P) == \
                oracle.sum_slice(f, j, n - 1, k0, k1, P, 8)[0], (f, j, n, k0, k1, P)


def test_long_runs_carry_the_digit_sums():
    # a lane carries its per-position digit sums every 120 terms and adds
    # them to its limbs at the end of its run: runs of 512 (one workgroup per
    # CU, run cap 4096) take four carry steps each
    saved = pb.get_tuning(1)
    try:
        pb.set_tuning(1, 1, 4096)
        f = pb.BELLARD
        rows, step, _ = oracle.series_table(f)
        s, c, a, b = rows[3]
        k0 = (2 ** 40 - b) // a + 12345
        k1 = k0 + 512 * 256 * 256 * 4 + 777
        n = step * k1 + 10 ** 7
        assert gpu_slice(f, 3, n, k0, k1, 64) == oracle.sum_slice(f, 3, n - 1, k0, k1, 64, 8)[0]
    finally:
        pb.set_tuning(1, *saved)


def test_slices_at_the_largest_moduli():
    # the last indices whose modulus is below the 2^54 limit (class 62's top),
    # with exponents near 2^61; one index further is refused
    rng = random.Random(54)
    for f in FORMULAS:
        rows, step, _ = oracle.series_table(f)
        for j, (s, c, a, b) in enumerate(rows):
            k1 = (2 ** 54 - 1 - b) // a + 1          # a (k1 - 1) + b < 2^54
            n = 2 ** 61 + rng.randrange(10 ** 6)
            for k0 in (k1 - 1, k1 - rng.randrange(2, 3000)):
                P = rng.choice([64, 320, 1088])
                assert gpu_slice(f, j, n, k0, k1, P) == \
                    oracle.sum_slice(f, j, n - 1, k0, k1, P, 8)[0], (f, j, k0, k1, P)
            with pytest.raises(pb.PiError):
                gpu_slice(f, j, n, k1, k1 + 1, 64)


def test_slices_large_moduli():
    # moduli near 2^40 (n = 10^12) and near 2^50 (n = 2*10^15), ragged lengths
    rng = random.Random(17)
    for n in (10 ** 12, 10 ** 12 + 1, 2 * 10 ** 15 - 3):
        for f in FORMULAS:
            rows, step, _ = oracle.series_table(f)
            for j in range(len(rows)):
                K = (n - 1 + rows[j][1]) // step + 1
                k0 = rng.randrange(0, K - 70_000)
                k1 = k0 + rng.randrange(1, 70_000)
                P = rng.choice([64, 320, 1088])
                assert gpu_slice(f, j, n, k0, k1, P) == \
                    oracle.sum_slice(f, j, n - 1, k0, k1, P, 8)[0], (n, f, j, k0, k1, P)


def test_slices_with_head_and_tail_and_empty():
    rng = random.Random(23)
    for f in FORMULAS:
        rows, step, _ = oracle.series_table(f)
        for j in range(len(rows)):
            n = rng.randrange(1, 50_000)
            K = max(0, (n - 1 + rows[j][1]) // step + 1)
            P = rng.choice([1, 63, 64, 65, 320, 1088])
            for k0, k1 in ((0, 0), (K, K), (0, K), (K, K + 500), (max(0, K - 40), K + 40),
                           (0, 2 ** 63), (K + 10 ** 6, K + 10 ** 6 + 5)):
                assert gpu_slice(f, j, n, k0, k1, P) == \
                    oracle.sum_slice(f, j, n - 1, k0, k1, P)[0], (f, j, n, k0, k1, P)


def test_partition_invariance():
    rng = random.Random(31)
    n, P = 3_000_001, 320
    for f in FORMULAS:
        S, _, _ = gpu_extract(f, n, 256, P)
        rows, step, _ = oracle.series_table(f)
        tot = 0
        for j in range(len(rows)):
            end = (n - 1 + rows[j][1] + P) // step + 2
            cuts = sorted(rng.sample(range(1, end), 9))
            for lo, hi in zip([0] + cuts, cuts + [end]):
                tot += gpu_slice(f, j, n, lo, hi, P)
        assert tot % 2 ** P == S


def test_deterministic_repeat():
    a = gpu_extract(pb.BELLARD, 12_345_679, 256, 320)
    b = gpu_extract(pb.BELLARD, 12_345_679, 256, 320)
    assert a == b


@pytest.mark.parametrize("m", [9, 10, 11])
def test_table_2_2_rows(m):
    row = [r for r in read_golden("table_2_2.txt") if r[0] == str(m)][0]
    S, N, cert = gpu_extract(pb.BELLARD, int(row[1]), 256, 320)
    assert cert
    assert S >> 64 == hex_bits(row[3], 256)


def test_bbp_and_bellard_agree_at_n1e10():
    a = gpu_extract(pb.BELLARD, 10 ** 10, 256, 320)
    b = gpu_extract(pb.BBP, 10 ** 10, 256, 320)
    assert a[2] and b[2]
    assert a[0] >> 64 == b[0] >> 64
    # Table 2.2's row m = 10 starts at 10^10 + 1: our bits after the first
    row = [r for r in read_golden("table_2_2.txt") if r[0] == "10"][0]
    assert (a[0] >> 64) & ((1 << 255) - 1) == hex_bits(row[3], 255)


def test_table_2_2_row_m12_full_size():
    # the full n = 10^12 + 1 query (7*10^11 head terms) in the launch
    # configuration the benchmark times; pinned by the paper's printed row
    row = [r for r in read_golden("table_2_2.txt") if r[0] == "12"][0]
    S, N, cert = gpu_extract(pb.BELLARD, int(row[1]), 256, 320)
    assert cert
    assert S >> 64 == hex_bits(row[3], 256)
    head = pb.head_terms(pb.BELLARD, int(row[1]))
    assert head == 700_000_000_002
    assert head < N <= head + 7 * (320 // 10 + 2)


@pytest.mark.parametrize("m", [9, 10, 11, 12])
def test_table_2_2_rows_all_printed_bits(m):
    # the paper's wide rows (1000, 1000, 996 and 1000 bits) at P = 1088: 17
    # limbs; m = 12 sums 7*10^11 head terms through the 24-digit binary64
    # division
    row = [r for r in read_golden("table_2_2.txt") if r[0] == str(m)][0]
    n, nbits = int(row[1]), int(row[2])
    S, N, cert = gpu_extract(pb.BELLARD, n, nbits, 1088)
    assert cert
    assert S >> (1088 - nbits) == hex_bits(row[3], nbits)


def test_results_do_not_depend_on_launch_shape():
    # the chunk partition changes with the launch shape; the sums must not
    saved = {L: pb.get_tuning(L) for L in (2, 5)}
    try:
        ref = {q: gpu_extract(*q) for q in ((pb.BELLARD, 3 * 10 ** 8 + 7, 256, 320),
                                            (pb.BBP, 2 * 10 ** 8 + 1, 64, 128))}
        for wg, cap in ((1, 1), (3, 7), (16, 128), (0, 64)):
            for L in (2, 5):
                pb.set_tuning(L, wg, cap)
            for q, want in ref.items():
                assert gpu_extract(*q) == want, (wg, cap, q)
    finally:
        for L, (wg, cap) in saved.items():
            pb.set_tuning(L, wg, cap)
