// Device integer arithmetic for one BBP-type term on gfx950.
//
// A head term (E >= 0) of eq (3.3) in Sze (2010) needs 2^E mod M and then a
// P-bit division r*2^P/M. Both are done without any division instruction:
//
//  * modular exponentiation (section 4.2 names Montgomery's method for large
//    moduli): a left-to-right ladder over exponent windows. In the integer
//    classes each step is one Montgomery reduction of x^2 * 2^b, so the
//    doubling for a 1 bit costs a shift, not a multiplication, and the
//    ladder's target exponent is chosen so that the Montgomery form of its
//    result is already s = 2^(E+64L) mod M. In the binary64 class the
//    residues are plain (2^E mod M itself) and each step is exact fp64
//    arithmetic.
//  * division, integer classes: with s = r*2^(64L) mod M, the quotient
//    t = floor(r*2^(64L)/M) satisfies t*M = r*2^(64L) - s, so
//    t = -s * M^-1 mod 2^(64L). That is an exact (Hensel) division, limb by
//    limb from the bottom, using the same -M^-1 mod 2^64 the Montgomery
//    reduction needs. Truncation to P bits: floor(t / 2^(64L-P)) =
//    floor(r*2^P/M), so the P-bit term, left-aligned in L limbs, is t with its
//    low 64L-P bits cleared.
//  * division, binary64 class: schoolbook long division of r 2^P by M from
//    the top, in signed digits of up to 46 bits, each one exact fp64 FMA
//    rounding and one exact fp64 FMA remainder; a lane sums its terms' digits
//    per position in doubles and turns the sums into limbs once per run.
//
// Modulus classes keep the instruction count down:
//  * class 32 (M < 2^29): R = 2^32, residues kept below 2M;
//  * binary64 (2^29 <= M < 2^51): plain (not Montgomery) residues held
//    exactly in doubles; a squaring is six full-rate fp64 instructions
//    against sixteen integer ones for the same modulus in class 62, exponent
//    windows of up to four bits cost two more per window, and from 2^48
//    five-bit windows apply their digit after the squarings, five more;
//  * class 62 (2^51 <= M < 2^54): R = 2^62, residues in two 31-bit digits,
//    kept below 8M;
//  * R = 2^64 with residues below 2M (M < 2^60): the few tail terms.
// v_mad_u64_u32 issues at full rate on gfx950, so the integer classes are
// written in plain 64-bit C and the compiler emits mad chains.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pibbp {

// ---- binary64 residues, 2^29 <= M < 2^51 -----------------------------------
//
// A residue is an integer-valued double x with |x| < M (signed, not reduced).
// One step computes y = 2^d x^2 - qM:
//   H + Lo = x (2^d x) exactly (H the rounded product, Lo its error, from an
//   FMA), q = rint(H * inv) with inv within 2^-51 of 1/M relatively, and
//   y = (H - qM) + Lo, where the FMA gives H - qM exactly (an integer below
//   2^53 in magnitude) and the last sum is exact for the same reason.
// Bound: |H/M - q| <= 1/2 + (H/M)(2^-51 + 2^-53) and |Lo| <= 2^-53 H, so
// |y| <= M/2 + 3 * 2^-52 * 2^d * M^2, which is below M while
// 2^d M <= 2^52 / 6 (about 2^49.4). Four-bit windows (d <= 15) are therefore
// exact for M < 2^34 and three-bit windows (d <= 7) for M < 2^42.
//
// From 2^42 the reciprocal is tighter: one Newton step from the previous
// modulus's reciprocal (at most 2^-37.7 away) leaves e^2 + 2^-53 with e^2 below
// 2^-75, so |y| <= M/2 + kappa H with kappa = 3 * 2^-53 (inv, the rounding of
// H inv, and Lo each 2^-53). Two-bit windows then keep |x| <= 0.75 M below
// 2^48: from 0.75 M the first squaring gives at most 0.553 M and the second
// (d <= 3) at most 0.73 M. From 2^48 to 2^51 a window is five plain
// squarings and then its digit on its own (scale_f64): from
// |x| <= M (1/2 + 2^-20) the squarings give at most 0.69, 0.86, 1.05, 1.33 and
// 1.82 M (every value below 2^53, so still exact), and 2^d y with d <= 31 is
// reduced by one rounded quotient (below 2^33) back to |x| <= M (1/2 + 2^-20).

// One Newton step toward 1/m from r: relative error e becomes e^2 + 2^-53.
// From 1/(M - 2a), at most 2^-26.6 away for M >= 2^31 and a <= 10, one step
// lands within 2^-52.2; from 2^29 (at most 2^-24.6 away) two steps do.
__device__ __forceinline__ double recip_step(double m, double r) {
#pragma clang fp contract(off)
  const double e = __builtin_fma(-m, r, 1.0);
  return __builtin_fma(r, e, r);
}

// 1/m to within 2^-53 (1 + 2^-20) from the hardware reciprocal: three steps
// leave any seed error below 2^-13 far below the final rounding.
__device__ __forceinline__ double recip_f64(double m) {
  return recip_step(m, recip_step(m, recip_step(m, __builtin_amdgcn_rcp(m))));
}

// y = 2^d x^2 mod M, |y| < M (bounds above).
__device__ __forceinline__ double sqr_f64(double x, int d, double M, double inv) {
#pragma clang fp contract(off)
  const double xs = __builtin_amdgcn_ldexp(x, d);
  const double h = x * xs;
  const double lo = __builtin_fma(x, xs, -h);
  const double q = __builtin_rint(h * inv);
  return __builtin_fma(-q, M, h) + lo;
}

__device__ __forceinline__ double sqr_f64(double x, double M, double inv) {
#pragma clang fp contract(off)
  const double h = x * x;
  const double lo = __builtin_fma(x, x, -h);
  const double q = __builtin_rint(h * inv);
  return __builtin_fma(-q, M, h) + lo;
}

// A window's digit applied on its own: 2^d y - rint(2^d y inv) M. For
// |y| <= 1.82 M, M < 2^51 and d <= 31, 2^d y / M is below 2^33 in magnitude
// and 2^d y inv is within 2^-20 of it, so the result is exact and at most
// M (1/2 + 2^-20) in magnitude. Five instructions with the digit's
// extraction.
__device__ __forceinline__ double scale_f64(double y, int d, double M, double inv) {
#pragma clang fp contract(off)
  const double ys = __builtin_amdgcn_ldexp(y, d);
  const double q = __builtin_rint(ys * inv);
  return __builtin_fma(-q, M, ys);
}

// 2^v mod M, |result| < M, for v < 64 and M >= 2^29: the error term
// 2^v (2^-51 + 2^-53) is below 2^13, far under M/2.
__device__ __forceinline__ double pow2_f64(uint32_t v, double M, double inv) {
#pragma clang fp contract(off)
  const double p = __builtin_amdgcn_ldexp(1.0, (int)v);
  const double q = __builtin_rint(p * inv);
  return __builtin_fma(-q, M, p);
}

// -M^-1 mod 2^32, M odd. (3M) xor 2 is an inverse to 5 bits; each Newton step
// x <- x(2 - Mx) doubles the number of correct low bits (5, 10, 20, 40).
__device__ __forceinline__ uint32_t neg_inv32(uint32_t m) {
  uint32_t x = (3u * m) ^ 2u;
  x *= 2u - m * x;
  x *= 2u - m * x;
  x *= 2u - m * x;
  return 0u - x;
}

// -M^-1 mod 2^64, M odd: one more Newton step from the 32-bit inverse.
__device__ __forceinline__ uint64_t neg_inv64(uint64_t m) {
  uint64_t x = (uint32_t)(0u - neg_inv32((uint32_t)m));
  x *= 2u - m * x;
  return 0u - x;
}

__device__ __forceinline__ int bitlen64(uint64_t x) { return x ? 64 - __clzll(x) : 0; }
__device__ __forceinline__ int bitlen32(uint32_t x) { return x ? 32 - __clz(x) : 0; }

// ---- class 64: R = 2^64, lazy residues in [0, 2M), M < 2^60 --------------

// Montgomery reduction of x^2 * 2^b: returns y == x^2 2^b 2^-64 (mod M),
// y < 2M, for x < 2M, b in {0, 1}. Since x^2 2^b + qM == 0 (mod 2^64), the
// low halves sum to exactly 2^64 unless x^2 2^b == 0 (mod 2^64), which gives
// the carry (lo != 0). Bound: y < 8M^2/2^64 + M + 1 <= 2M for M < 2^60.
__device__ __forceinline__ uint64_t sqr_redc64(uint64_t x, uint32_t b, uint64_t M, uint64_t mp) {
  uint64_t y = x << b;
  uint64_t lo = x * y;
  uint64_t hi = __umul64hi(x, y);
  uint64_t q = lo * mp;
  uint64_t h = __umul64hi(q, M);
  return hi + h + (lo != 0u ? 1u : 0u);
}

// 2^64 mod M (the Montgomery form of 1), M odd, 3 <= M < 2^60: start from
// 2^bl - M == 2^bl (mod M), bl = bit length of M, then double 64 - bl times.
__device__ __forceinline__ uint64_t mont_one64(uint64_t M) {
  int bl = bitlen64(M);
  uint64_t c = (1ull << bl) - M;
  for (int i = bl; i < 64; ++i) {
    c <<= 1;
    c = c >= M ? c - M : c;
  }
  return c;
}

// ---- class 62: R = 2^62, residues in two 31-bit digits, M < 2^54 ---------
//
// x = d0 + d1 2^31 with d0 < 2^31. Every partial product is below 2^63 and
// every column sum below 2^64, so no carry ever has to be tracked: the
// reduction digit u == (column mod 2^31) * (-M^-1) (mod 2^31) clears the low
// 31 bits of its column, and the column shifted right by 31 feeds the next.
// u is used as the full 32-bit product (not reduced mod 2^31): only its
// residue mod 2^31 matters for the cancellation, and the extra multiple of
// 2^31 M it adds is covered by the bounds below.

constexpr uint32_t kMask31 = 0x7fffffffu;

// a * b + c with the 64-bit addend fused into one v_mad_u64_u32 (the carry out
// is not needed: every sum here is below 2^64).
__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t d, cc;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(cc) : "v"(a), "v"(b), "v"(c));
  (void)cc;
  return d;
}

// x <- 2^b * REDC(x^2) == 2^b x^2 2^-62 (mod M), for x < 8M, b in {0, 1},
// odd M < 2^54 with digits m0 < 2^31, m1 < 2^23 and p == -M^-1 (mod 2^31).
// Bounds: d1 < 2^26, u0, u1 < 2^32; c0 < 2^62 + 2^63, c1 < 2^63.2,
// c2 < 2^56. The reduction multiplier mu = u0 + u1 2^31 is below
// 2^63 + 2^32, so REDC(x^2) < 64M^2/2^62 + 2.0001M < 2.26M and after the
// doubling x < 4.52M < 8M again.
__device__ __forceinline__ void sqr_redc62(uint32_t &d0, uint32_t &d1, uint32_t b, uint32_t m0,
                                           uint32_t m1, uint32_t p) {
  uint64_t c0 = (uint64_t)d0 * d0;
  const uint32_t u0 = (uint32_t)c0 * p;
  c0 = mad64(u0, m0, c0);
  uint64_t c1 = mad64(d0, d1 << 1, c0 >> 31);
  c1 = mad64(u0, m1, c1);
  const uint32_t u1 = (uint32_t)c1 * p;
  c1 = mad64(u1, m0, c1);
  uint64_t c2 = mad64(d1, d1, c1 >> 31);
  c2 = mad64(u1, m1, c2);
  c2 <<= b;
  d0 = (uint32_t)c2 & kMask31;
  d1 = (uint32_t)(c2 >> 31);
}

// floor(2^62 / M) for 2^31 <= M < 2^54, by restoring long division: the
// quotient has at most 32 bits, and bit s is tried only while M 2^s stays
// below 2^64.
__device__ __forceinline__ uint32_t div_2_62(uint64_t M) {
  const int room = 63 - bitlen64(M);  // largest s with M << s < 2^63
  uint64_t r = 1ull << 62;
  uint32_t q = 0;
  for (int s = 31; s >= 0; --s) {
    if (s <= room) {
      const uint64_t ms = M << s;
      if (r >= ms) {
        r -= ms;
        q |= 1u << s;
      }
    }
  }
  return q;
}

// ---- class 32: R = 2^32, residues in [0, 2M), M < 2^29 -------------------

// x^2 2^-32 mod M, lazily (x < 2M, M < 2^30): T = x^2 < 4M^2, so
// (T + qM) / 2^32 < 4M^2 / 2^32 + M < 2M. Three instructions.
__device__ __forceinline__ uint32_t sqr_redc32_plain(uint32_t x, uint32_t M, uint32_t mp) {
  const uint64_t T = (uint64_t)x * x;
  const uint32_t q = (uint32_t)T * mp;
  return (uint32_t)((T + (uint64_t)q * M) >> 32);
}

// With a window digit d: x^2 2^d 2^-32 mod M stays below 2M while
// 2^(d+2) M < 2^32, i.e. d <= 3 for M < 2^27 and d <= 7 for M < 2^23, and
// x 2^d < 2^31 then fits a word.
__device__ __forceinline__ uint32_t sqr_redc32_digit(uint32_t x, uint32_t d, uint32_t M,
                                                     uint32_t mp) {
  const uint64_t T = (uint64_t)x * (x << d);
  const uint32_t q = (uint32_t)T * mp;
  return (uint32_t)((T + (uint64_t)q * M) >> 32);
}

// floor(2^32 / M) for 2^22 <= M < 2^29 (restoring division; at most 11
// quotient bits).
__device__ __forceinline__ uint32_t div_2_32(uint32_t M) {
  uint64_t r = 1ull << 32;
  uint32_t q = 0;
  for (int s = 10; s >= 0; --s) {
    const uint64_t ms = (uint64_t)M << s;
    if (r >= ms) {
      r -= ms;
      q |= 1u << s;
    }
  }
  return q;
}

// 2^32 mod M, M odd, 3 <= M < 2^31.
__device__ __forceinline__ uint32_t mont_one32(uint32_t M) {
  int bl = bitlen32(M);
  uint32_t c = (1u << bl) - M;
  for (int i = bl; i < 32; ++i) {
    c <<= 1;
    c = min(c, c - M);
  }
  return c;
}

// ---- limb vectors ---------------------------------------------------------

// L-limb add and negate mod 2^(64L), written on 32-bit halves so that the
// compiler emits one v_add_co / v_addc_co (v_sub_co / v_subb_co) carry chain,
// two instructions per limb.
template <int L>
__device__ __forceinline__ void add_limbs(uint64_t (&acc)[L], const uint64_t (&t)[L]) {
  unsigned int c = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const unsigned int lo = __builtin_addc((unsigned int)acc[i], (unsigned int)t[i], c, &c);
    const unsigned int hi =
        __builtin_addc((unsigned int)(acc[i] >> 32), (unsigned int)(t[i] >> 32), c, &c);
    acc[i] = ((uint64_t)hi << 32) | lo;
  }
}

template <int L>
__device__ __forceinline__ void neg_limbs(uint64_t (&x)[L]) {
  unsigned int c = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const unsigned int lo = __builtin_subc(0u, (unsigned int)x[i], c, &c);
    const unsigned int hi = __builtin_subc(0u, (unsigned int)(x[i] >> 32), c, &c);
    x[i] = ((uint64_t)hi << 32) | lo;
  }
}

// t = -s * M^-1 mod 2^(64L): the L-limb quotient floor(r 2^(64L) / M) when
// s = r 2^(64L) mod M (Hensel division, 64-bit limbs). h carries the part of
// the dividend not yet divided; it stays below M.
template <int L>
__device__ __forceinline__ void hensel64(uint64_t s, uint64_t M, uint64_t mp, uint64_t (&t)[L]) {
  uint64_t h = s;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint64_t ti = h * mp;
    h = __umul64hi(ti, M) + (h != 0u ? 1u : 0u);
    t[i] = ti;
  }
}

// x >> 1 as one 64-bit shift whose low register is then reused as lo32:
// written out, the compiler recomputes that low word with an extra funnel
// shift from the unshifted value.
__device__ __forceinline__ uint64_t shr1_64(uint64_t x) {
  uint64_t y;
  asm("v_lshrrev_b64 %0, 1, %1" : "=v"(y) : "v"(x));
  return y;
}

// The same quotient from 32-bit digits for any odd M < 2^62, with only
// mp32 = -M^-1 mod 2^32. Digit u = lo32(h) * mp32 makes h + uM divisible by
// 2^32. With M = m1 2^31 + m0 (m0 < 2^31): A = u m0 + h stays below 2^64 and
// is divisible by 2^31, and h' = (h + uM) / 2^32 = (u m1 + A / 2^31) / 2.
// h stays below M. Each digit is a multiply, two full-rate multiply-adds and
// two 64-bit shifts, all on aligned register pairs.
template <int L>
__device__ __forceinline__ void hensel_d32(uint64_t s, uint64_t M, uint32_t mp32,
                                           uint64_t (&t)[L]) {
  const uint32_t m0 = (uint32_t)M & 0x7fffffffu, m1 = (uint32_t)(M >> 31);
  uint64_t h = s;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint32_t dg[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t u = (uint32_t)h * mp32;
      const uint64_t A = mad64(u, m0, h);
      h = shr1_64(mad64(u, m1, A >> 31));
      dg[j] = u;
    }
    t[i] = ((uint64_t)dg[1] << 32) | dg[0];
  }
}

// The same with 32-bit digits, for class-32 moduli (M < 2^31,
// mp32 = -M^-1 mod 2^32). Digit u = h * mp32 makes h + uM divisible by 2^32;
// h + uM < 2^63, so one v_mad_u64_u32 forms it exactly and its high word is
// the next h, again below M: two instructions per digit.
template <int L>
__device__ __forceinline__ void hensel32(uint32_t s, uint32_t M, uint32_t mp32, uint64_t (&t)[L]) {
  uint32_t h = s;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint32_t lo = h * mp32;
    h = (uint32_t)(mad64(lo, M, h) >> 32);
    const uint32_t hi = h * mp32;
    if (i + 1 < L) h = (uint32_t)(mad64(hi, M, h) >> 32);
    t[i] = ((uint64_t)hi << 32) | lo;
  }
}

// Masks that clear the low 64L-P bits of an L-limb value (P <= 64L); built
// once per chunk, applied to every term with one AND per 32-bit word.
// Limbs of a kernel limb class L that can hold cleared bits: a query uses the
// smallest class with 64L >= P, so 64L - P < 64 (L - previous class), and only
// that many low limbs need a mask (classes 1..6, 8, 12, 17).
constexpr int masked_limbs(int L) { return L == 8 ? 2 : L == 12 ? 4 : L == 17 ? 5 : 1; }

template <int L>
__device__ __forceinline__ void low_masks(uint32_t P, uint64_t (&m)[L]) {
  const uint32_t z = 64u * L - P;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint32_t lo = 64u * i;
    m[i] = z >= lo + 64u ? 0ull : (z > lo ? ~0ull << (z - lo) : ~0ull);
  }
}

// Apply the masks of the low limbs that can need one (see masked_limbs).
template <int L>
__device__ __forceinline__ void apply_masks(uint64_t (&t)[L], const uint64_t (&m)[L]) {
#pragma unroll
  for (int i = 0; i < masked_limbs(L); ++i) t[i] &= m[i];
}

// Clear the low 64L-P bits (any P <= 64L), for the few terms outside the hot
// loop.
template <int L>
__device__ __forceinline__ void clip_low(uint64_t (&t)[L], uint32_t P) {
  uint64_t m[L];
  low_masks<L>(P, m);
#pragma unroll
  for (int i = 0; i < L; ++i) t[i] &= m[i];
}

// ---- binary64 long division of one term --------------------------------------
//
// The P-bit term floor(r 2^P / M) of a residue r (integer-valued double,
// |r| < M) in signed digits, most significant first: digit d (d = 0 the
// lowest) holds bits [dB, dB + B) of the term; the top one, d = ne - 1 with
// ne = ceil(P / B), holds the remaining bt = P - (ne - 1)B bits. From a
// remainder y, a digit of b bits is q = rint(y 2^b / M) and the next remainder
// y 2^b - qM:
//   ys = y 2^b (exact); fma(ys, inv, C) with C = 1.5 * 2^52 rounds the exact
//   product ys * inv to an integer in one step (spacing 1 in [2^52, 2^53),
//   and |ys inv| <= 2^46 (1 + 2^-50) < 2^51), so q = that - C;
//   y' = fma(-q, M, ys) is exact: its value is an integer below M.
// With inv within 2^-52 of 1/M relatively, |ys inv - ys/M| <= 2^b 2^-52 <= 2^-6
// (b <= 46), so |y'| <= M (1/2 + 2^-6) and every digit after the top one has
// |q| <= 2^(B-1) + 2^(B-6) + 1; the top one |q| <= 2^bt + 1.
// After the last digit r 2^P = M * sum_d q_d 2^(dB) + y_N with |y_N| < M, so
// floor(r 2^P / M) = sum_d q_d 2^(dB) - [y_N < 0]. A negative r gives the term
// of r + M, floor((r + M) 2^P / M) = floor(r 2^P / M) + 2^P, up to that 2^P,
// which the sum mod 2^P drops.
//
// A lane sums its terms' digits per position in doubles. Every kFpCarryTerms
// terms the sums are carried upward until each lies in [0, 2^B) (the carry
// out of the top position lands at or above bit N B >= P and is dropped);
// from there 120 more digits of |q| <= 2^46 + 1 keep every sum below
// 121 * 2^46 + 120 < 2^53, so exact. At the end of the run the sums go into
// the lane's limbs. B <= 46 bits per digit, as few digits per limb count L as
// cover 64L bits: N B >= 64L >= P.
constexpr uint32_t kFpCarryTerms = 120;
constexpr int fp_digits(int L) { return (64 * L + 45) / 46; }
constexpr int fp_digit_bits(int L) { return (64 * L + fp_digits(L) - 1) / fp_digits(L); }

// Digits of one term from y = r into the per-position sums A; nneg counts the
// terms whose last remainder is negative. bits[d] is B below the top digit,
// bt for it and 0 above it (wave-uniform): a 0-bit digit is rint(y / M),
// whose weight 2^P vanishes mod 2^P, as does A_d 2^(dB) for those d.
template <int N>
__device__ __forceinline__ void fp_term_digits(double y, double M, double inv,
                                               const int (&bits)[N], double (&A)[N],
                                               uint32_t &nneg) {
#pragma clang fp contract(off)
  constexpr double C = 0x1.8p52;
#pragma unroll
  for (int d = N - 1; d >= 0; --d) {
    const double ys = __builtin_amdgcn_ldexp(y, bits[d]);
    const double q = __builtin_fma(ys, inv, C) - C;
    y = __builtin_fma(-q, M, ys);
    A[d] += q;
  }
  nneg += y < 0.0 ? 1u : 0u;
}

// The digit sizes for P bits: ne = ceil(P / B) digits, the top one
// P - (ne - 1)B bits, and 0 bits for positions from ne up.
template <int N, int B>
__device__ __forceinline__ void fp_digit_sizes(uint32_t P, int (&bits)[N]) {
  const int ne = (int)((P + B - 1u) / B), bt = (int)P - (ne - 1) * B;
#pragma unroll
  for (int d = 0; d < N; ++d)
    bits[d] = __builtin_amdgcn_readfirstlane(d < ne - 1 ? B : d == ne - 1 ? bt : 0);
}

// The carry step: subtracts nneg from the lowest position, then brings every
// A_d into [0, 2^B) by moving floor(A_d / 2^B) up one position (each carry
// is at most 122 in magnitude, so A_{d+1} plus it stays below 2^53); the
// carry out of the top position is dropped.
template <int N, int B>
__device__ __forceinline__ void fp_carry_digits(double (&A)[N], uint32_t &nneg) {
#pragma clang fp contract(off)
  constexpr double kTwoB = (double)(1ull << B);
  A[0] -= (double)nneg;
  nneg = 0;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    const double c = __builtin_floor(__builtin_amdgcn_ldexp(A[d], -B));
    A[d] = __builtin_fma(-c, kTwoB, A[d]);
    if (d + 1 < N) A[d + 1] += c;
  }
}

// Adds sum_d A_d 2^(dB) - nneg, mod 2^P, at bit 64L - P of the L-limb sum,
// and clears A and nneg. After the carry step the digits occupy disjoint bit
// fields and are packed with shifts known at compile time; the packed value
// moves up by 64L - P bits (fewer than 64 masked_limbs(L), as a query uses
// the smallest limb class that holds P), and bits from 64L up fall away.
template <int L>
__device__ __forceinline__ void fp_digits_to_limbs(double (&A)[fp_digits(L)], uint32_t &nneg,
                                                   uint32_t P, uint64_t (&sum)[L]) {
#pragma clang fp contract(off)
  constexpr int N = fp_digits(L), B = fp_digit_bits(L);
  fp_carry_digits<N, B>(A, nneg);
  uint64_t V[L + 1];
#pragma unroll
  for (int i = 0; i <= L; ++i) V[i] = 0;
#pragma unroll
  for (int d = 0; d < N; ++d) {
    const uint64_t u = (uint64_t)__double_as_longlong(A[d] + 0x1p52) & ((1ull << 52) - 1u);
    const int pos = d * B, li = pos >> 6, off = pos & 63;
    V[li] |= u << off;
    if (off + B > 64) V[li + 1] |= u >> (64 - off);
  }
  const uint32_t z = 64u * L - P, zl = z >> 6, zb = z & 63u;
  uint64_t Wl[L];
#pragma unroll
  for (int j = 0; j < L; ++j) Wl[j] = V[j];
#pragma unroll
  for (int c = 1; c < masked_limbs(L); ++c)
    if (zl == (uint32_t)c) {
#pragma unroll
      for (int j = L - 1; j >= 0; --j) Wl[j] = j >= c ? V[j - c] : 0ull;
    }
  uint64_t T[L];
#pragma unroll
  for (int j = 0; j < L; ++j)
    T[j] = zb ? (Wl[j] << zb) | (j ? Wl[j - 1] >> (64u - zb) : 0ull) : Wl[j];
  add_limbs<L>(sum, T);
#pragma unroll
  for (int d = 0; d < N; ++d) A[d] = 0.0;
  nneg = 0;
}

}  // namespace pibbp
