/*
 * A test program for the oracle built with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitized.py): it calls every oracle entry
 * point at the edges of its arguments (one-bit and 1088-bit sums, the limits
 * of the word arithmetic, tail terms with modulus 1, empty and tail-only
 * ranges, several threads) and prints each result as one text line, which
 * the test compares with the ordinary build of the same functions.
 */
#include <inttypes.h>
#include <stdio.h>
#include <stdlib.h>

#include "pio.h"

static void put_words(const char *tag, const uint32_t *x, uint32_t nw) {
  printf("%s", tag);
  for (uint32_t i = nw; i-- > 0;) printf(" %08" PRIx32, x[i]);
  printf("\n");
}

static uint32_t nwords(uint32_t bits) { return (bits + 31u) / 32u; }

int main(void) {
  static const uint32_t Ps[] = {1, 2, 31, 32, 33, 63, 64, 65, 320, 1087, 1088};
  const int nP = (int)(sizeof Ps / sizeof Ps[0]);
  uint32_t *buf = (uint32_t *)calloc(64, sizeof(uint32_t));
  char tag[160];

  static const uint64_t pe[][2] = {{0, 1}, {5, 1}, {0, 7}, {1, 3}, {63, 2305843009213693951ull},
                                   {1000000000000000ull, 1125899906842625ull},
                                   {4611686018427387903ull, 18014398509481983ull}};
  for (size_t i = 0; i < sizeof pe / sizeof pe[0]; ++i)
    printf("pow %" PRIu64 " %" PRIu64 " %" PRIu64 "\n", pe[i][0], pe[i][1],
           pio_pow2mod(pe[i][0], pe[i][1]));

  for (int f = 0; f < 2; ++f) {
    const int J = f ? 7 : 4;
    for (int j = 0; j < J; ++j)
      for (int ip = 0; ip < nP; ++ip) {
        const uint32_t P = Ps[ip];
        /* head terms, the last head index, tail terms including modulus 1 at k = 0 */
        static const uint64_t dk[][2] = {{0, 0}, {1, 0}, {9, 0}, {200, 3}, {200, 20}, {200, 25},
                                         {1000000, 99999}, {2000000000000000ull, 199999999999999ull}};
        for (size_t c = 0; c < sizeof dk / sizeof dk[0]; ++c) {
          if (pio_term(f, j, dk[c][0], dk[c][1], P, buf) != 0) return 2;
          snprintf(tag, sizeof tag, "term %d %d %" PRIu64 " %" PRIu64 " %u", f, j, dk[c][0],
                   dk[c][1], P);
          put_words(tag, buf, nwords(P));
        }
        static const uint64_t rk[][3] = {{500, 0, 0}, {500, 10, 10}, {500, 0, 200},
                                         {500, 40, 60}, {500, 120, 1000}, {3, 0, 1000}};
        for (size_t c = 0; c < sizeof rk / sizeof rk[0]; ++c)
          for (int nt = 1; nt <= 4; nt += 3) {
            uint64_t N = 0;
            if (pio_sum_slice(f, j, rk[c][0], rk[c][1], rk[c][2], P, buf, &N, nt) != 0) return 3;
            snprintf(tag, sizeof tag, "slice %d %d %" PRIu64 " %" PRIu64 " %" PRIu64 " %u %d %" PRIu64,
                     f, j, rk[c][0], rk[c][1], rk[c][2], P, nt, N);
            put_words(tag, buf, nwords(P));
          }
      }
    static const uint64_t ns[] = {1, 2, 3, 9, 1000, 100001};
    for (size_t c = 0; c < sizeof ns / sizeof ns[0]; ++c)
      for (int ip = 0; ip < nP; ++ip) {
        const uint32_t P = Ps[ip];
        const uint32_t ws[] = {1, P > 64 ? P - 64 : 1, P};
        for (int iw = 0; iw < 3; ++iw) {
          uint64_t N = 0;
          int32_t cert = -1;
          if (pio_extract(f, ns[c], ws[iw], P, buf, &N, &cert, 3) != 0) return 4;
          snprintf(tag, sizeof tag, "extract %d %" PRIu64 " %u %u %" PRIu64 " %d", f, ns[c],
                   ws[iw], P, N, (int)cert);
          put_words(tag, buf, nwords(P));
        }
      }
  }

  for (int ip = 0; ip < nP; ++ip) {
    const uint32_t P = Ps[ip];
    for (uint32_t i = 0; i < nwords(P); ++i) buf[i] = 0x9e3779b9u * (i + 1u) + P;
    if (P % 32u) buf[nwords(P) - 1] &= (1u << (P % 32u)) - 1u;
    static const uint64_t Bs[] = {0, 1, 7, 1000, 18446744073709551615ull};
    for (uint32_t w = 1; w <= P; w += (P < 70 ? 1 : 97))
      for (size_t b = 0; b < sizeof Bs / sizeof Bs[0]; ++b)
        printf("certify %u %u %" PRIu64 " %d\n", P, w, Bs[b], pio_certify(buf, P, w, Bs[b]));
  }

  static const uint32_t mb[] = {1, 31, 32, 33, 1000};
  for (size_t i = 0; i < sizeof mb / sizeof mb[0]; ++i) {
    const int ok = pio_machin(mb[i], buf);
    snprintf(tag, sizeof tag, "machin %u %d", mb[i], ok);
    put_words(tag, buf, nwords(mb[i]));
  }
  free(buf);
  return 0;
}
