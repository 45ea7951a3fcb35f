/*
 * pio.h -- the oracle: a plain, slow, CPU-only evaluation of BBP-type digit
 * extraction of pi (Sze, "The Two Quadrillionth Bit of pi is 0!", sections 1
 * and 3). TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke check
 * and the benchmark's CPU baseline can check the GPU library against an
 * independent implementation. It shares no code with the GPU library and
 * nothing in the product path may call it.
 *
 * Big integers here are little-endian arrays of uint32_t words.  A P-bit
 * value occupies ceil(P/32) words; bits at and above P are always zero.
 */
#ifndef PIO_H
#define PIO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PIO_BBP = 0, PIO_BELLARD = 1 };

/* Row of a series table: the series contributes
 *   sign * sum_k alt^k * 2^(d + c - step*k) / (a*k + b)
 * to 2^d * pi, with alt = -1 for Bellard's formula and +1 for BBP. */
typedef struct { int32_t sign, c; uint64_t a, b; } pio_series;

/* Copy the series table of `formula` into out[0..J-1]; returns J, or -1 for an
 * unknown formula. step and alt (+1 or -1) are written when non-NULL. */
int pio_series_table(int formula, pio_series *out, int32_t *step, int32_t *alt);

/* 2^e mod m by right-to-left square-and-multiply (m >= 1). */
uint64_t pio_pow2mod(uint64_t e, uint64_t m);

/* One term of series j at shift d (d = n-1) and index k, at P fraction bits:
 *   t = floor(2^P * frac(2^E / M)),  E = d + c - step*k,  M = a*k + b.
 * out: ceil(P/32) words. Returns 0, or -1 on bad arguments. */
int pio_term(int formula, int j, uint64_t d, uint64_t k, uint32_t P, uint32_t *out);

/* sum over k in [k0, k1) of sign_j * alt^k * t_{j,k}  mod 2^P  (out: ceil(P/32)
 * words). *nterms receives the number of indices summed before the series'
 * stop index (the first tail index whose t is 0), or NULL. */
int pio_sum_slice(int formula, int j, uint64_t d, uint64_t k0, uint64_t k1, uint32_t P,
                  uint32_t *out, uint64_t *nterms, int nthreads);

/* Whole extraction at 1-based bit position n: S = the P-bit sum over every
 * series (head and tail up to its stop index), N = number of indices summed,
 * certified = 1 when the guard window proves the top w bits of S equal bits
 * n .. n+w-1 of pi. S: ceil(P/32) words. */
int pio_extract(int formula, uint64_t n, uint32_t w, uint32_t P, uint32_t *S,
                uint64_t *N, int32_t *certified, int nthreads);

/* The certification test of pio_extract on its own (section 3.1, adapted to
 * truncated terms): S is a P-bit sum (ceil(P/32) words), B the error bound in
 * units of 2^-P. Returns 1 when every real number within B units of S
 * (exclusive, modulo 2^P) has the same top w bits as S, i.e. when
 * G >= B and G + B <= 2^(P-w) for the guard window G = S mod 2^(P-w);
 * 0 otherwise. Requires 1 <= w <= P and B < 2^64. */
int pio_certify(const uint32_t *S, uint32_t P, uint32_t w, uint64_t B);

/* floor(frac(pi) * 2^nbits) by Machin's formula; out: ceil(nbits/32) words.
 * Returns 0 when the guard bits prove every output bit, -1 otherwise. */
int pio_machin(uint32_t nbits, uint32_t *out);

#ifdef __cplusplus
}
#endif
#endif
