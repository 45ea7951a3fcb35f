/*
 * pio.c -- the oracle (test infrastructure only; see pio.h).
 *
 * What it computes (Sze 2010, section 3, eqs (3.1)-(3.3); Bellard's formula
 * (1.2); the BBP formula (1.1) in the odd-denominator form of (3.1)):
 *
 *   frac(2^d pi) = frac( sum_j sign_j sum_k alt^k 2^(d+c_j-step*k) / (a_j k + b_j) ).
 *
 * A term whose exponent E = d+c_j-step*k is >= 0 ("head", A_k of (3.3)) has
 * fractional part (2^E mod M)/M; a term with E < 0 ("tail", B_k of (3.3)) is
 * 2^E/M.  Every term is truncated to P fraction bits,
 *
 *   t = floor(2^P * frac(2^E / M)),
 *
 * and the signed terms are added modulo 2^P.  In each series the tail is cut
 * at its first term whose truncation is 0; every later tail term is smaller.
 *
 * Nothing here is tuned: modular exponentiation is right-to-left
 * square-and-multiply with a 128-bit product and '%', and t comes from
 * schoolbook long division of r*2^P by M, one 32-bit digit at a time.
 */
#include "pio.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- series tables ------------------------------------------------------ */

/* Bellard's formula (1.2): pi = sum_k (-1)^k 2^(-10k) * ( 2^2/(10k+1) - 1/(10k+3)
 * - 2^-4/(10k+5) - 2^-4/(10k+7) + 2^-6/(10k+9) - 2^-1/(4k+1) - 2^-6/(4k+3) ).
 * The power of two in front of each fraction becomes c. */
static const pio_series BELLARD[7] = {
    {+1, 2, 10, 1}, {-1, 0, 10, 3}, {-1, -4, 10, 5}, {-1, -4, 10, 7},
    {+1, -6, 10, 9}, {-1, -1, 4, 1}, {-1, -6, 4, 3},
};
/* The BBP formula as written in (3.1): the 8k+4 and 8k+6 denominators of (1.1)
 * are halved into 2k+1 and 4k+3 with an extra factor 2^-1. */
static const pio_series BBP[4] = {
    {+1, 2, 8, 1}, {-1, -1, 2, 1}, {-1, 0, 8, 5}, {-1, -1, 4, 3},
};

int pio_series_table(int formula, pio_series *out, int32_t *step, int32_t *alt) {
  const pio_series *tab;
  int J, st, al;
  if (formula == PIO_BELLARD) { tab = BELLARD; J = 7; st = 10; al = -1; }
  else if (formula == PIO_BBP) { tab = BBP; J = 4; st = 4; al = +1; }
  else return -1;
  if (out) memcpy(out, tab, sizeof(pio_series) * (size_t)J);
  if (step) *step = st;
  if (alt) *alt = al;
  return J;
}

/* ---- small big-integer helpers (little-endian uint32 words) -------------- */

static uint32_t nwords(uint32_t bits) { return (bits + 31u) / 32u; }

/* Clear every bit at or above position `bits`. */
static void clip(uint32_t *x, uint32_t nw, uint32_t bits) {
  for (uint32_t i = 0; i < nw; ++i) {
    uint32_t lo = 32u * i;
    if (lo >= bits) x[i] = 0;
    else if (bits - lo < 32u) x[i] &= (1u << (bits - lo)) - 1u;
  }
}

/* x = (x + y) mod 2^bits */
static void add_mod(uint32_t *x, const uint32_t *y, uint32_t nw, uint32_t bits) {
  uint64_t carry = 0;
  for (uint32_t i = 0; i < nw; ++i) {
    uint64_t s = (uint64_t)x[i] + y[i] + carry;
    x[i] = (uint32_t)s;
    carry = s >> 32;
  }
  clip(x, nw, bits);
}

/* x = (x - y) mod 2^bits */
static void sub_mod(uint32_t *x, const uint32_t *y, uint32_t nw, uint32_t bits) {
  uint64_t borrow = 0;
  for (uint32_t i = 0; i < nw; ++i) {
    uint64_t d = (uint64_t)x[i] - y[i] - borrow;
    x[i] = (uint32_t)d;
    borrow = (d >> 63) & 1u;
  }
  clip(x, nw, bits);
}

static int is_zero(const uint32_t *x, uint32_t nw) {
  for (uint32_t i = 0; i < nw; ++i)
    if (x[i]) return 0;
  return 1;
}

/* ---- the two arithmetic steps of a term ---------------------------------- */

uint64_t pio_pow2mod(uint64_t e, uint64_t m) {
  uint64_t result = 1 % m, base = 2 % m;
  while (e) {
    if (e & 1u) result = (uint64_t)((u128)result * base % m);
    base = (uint64_t)((u128)base * base % m);
    e >>= 1;
  }
  return result;
}

/* q = floor(r * 2^bits / m) for 0 <= r < m, by long division in base 2^32:
 * the dividend r*2^(32*nw) is consumed one zero digit at a time, and the
 * quotient is shifted down by the excess 32*nw - bits at the end, which is the
 * same floor because floor(floor(x)/2^s) = floor(x/2^s). */
static void div_frac(uint64_t r, uint64_t m, uint32_t bits, uint32_t *q, uint32_t nw) {
  uint32_t nd = nwords(bits);
  uint32_t *tmp = (uint32_t *)calloc(nd + 1, sizeof(uint32_t));
  u128 rem = r;
  for (uint32_t i = nd; i-- > 0;) {
    u128 cur = rem << 32;                 /* next digit of the dividend is 0 */
    tmp[i] = (uint32_t)(cur / m);
    rem = cur % m;
  }
  uint32_t s = 32u * nd - bits;           /* 0 <= s < 32 */
  memset(q, 0, sizeof(uint32_t) * nw);
  for (uint32_t i = 0; i < nd && i < nw; ++i) {
    uint64_t two = (uint64_t)tmp[i] | ((uint64_t)tmp[i + 1] << 32);
    q[i] = (uint32_t)(two >> s);
  }
  free(tmp);
}

static int term_at(const pio_series *sr, int32_t step, uint64_t d, uint64_t k, uint32_t P,
                   uint32_t *out) {
  uint32_t nw = nwords(P);
  int64_t E = (int64_t)d + sr->c - (int64_t)step * (int64_t)k;
  uint64_t M = sr->a * k + sr->b;
  memset(out, 0, sizeof(uint32_t) * nw);
  if (E >= 0) {
    /* head term A_k: (2^E mod M)/M */
    uint64_t r = pio_pow2mod((uint64_t)E, M);
    if (r) div_frac(r, M, P, out, nw);
  } else {
    /* tail term B_k: 2^E/M = 1/(2^-E M); its P-bit truncation is
     * floor(2^(P+E)/M), zero when P+E < 0 */
    int64_t bits = (int64_t)P + E;
    if (bits < 0) return 0;
    if (M == 1) {
      out[bits / 32] = 1u << (bits % 32);
    } else {
      div_frac(1, M, (uint32_t)bits, out, nw);
    }
  }
  return 0;
}

int pio_term(int formula, int j, uint64_t d, uint64_t k, uint32_t P, uint32_t *out) {
  pio_series tab[7];
  int32_t step;
  int J = pio_series_table(formula, tab, &step, NULL);
  if (J < 0 || j < 0 || j >= J || P == 0) return -1;
  return term_at(&tab[j], step, d, k, P, out);
}

/* ---- sums ---------------------------------------------------------------- */

typedef struct {
  pio_series sr;
  int32_t step, alt;
  uint64_t d, k0, k1;
  uint32_t P;
  uint32_t *acc;    /* ceil(P/32) words, zeroed by the caller */
  uint64_t nterms;  /* indices summed before the stop index */
} slice_job;

/* Plain loop over k in [k0, k1): add sign * alt^k * t. A tail index whose t
 * is zero is the stop index: nothing after it can be nonzero. */
static void *run_slice(void *arg) {
  slice_job *jb = (slice_job *)arg;
  uint32_t nw = nwords(jb->P);
  uint32_t *t = (uint32_t *)calloc(nw, sizeof(uint32_t));
  for (uint64_t k = jb->k0; k < jb->k1; ++k) {
    int64_t E = (int64_t)jb->d + jb->sr.c - (int64_t)jb->step * (int64_t)k;
    term_at(&jb->sr, jb->step, jb->d, k, jb->P, t);
    if (E < 0 && is_zero(t, nw)) break;
    int neg = (jb->sr.sign < 0) ^ (jb->alt < 0 && (k & 1u));
    if (neg) sub_mod(jb->acc, t, nw, jb->P);
    else add_mod(jb->acc, t, nw, jb->P);
    jb->nterms++;
  }
  free(t);
  return NULL;
}

/* Split [k0,k1) into nthreads pieces, sum each in its own thread, add the
 * partial sums. Additions mod 2^P commute, so the split changes nothing. The
 * stop rule applies only inside the tail, where t never increases with k, so
 * it is applied to the tail part in one piece. */
static int sum_range(const pio_series *sr, int32_t step, int32_t alt, uint64_t d, uint64_t k0,
                     uint64_t k1, uint32_t P, uint32_t *out, uint64_t *nterms, int nthreads) {
  uint32_t nw = nwords(P);
  memset(out, 0, sizeof(uint32_t) * nw);
  if (nterms) *nterms = 0;
  if (k1 <= k0) return 0;
  /* first tail index: smallest k with d + c - step*k < 0 */
  int64_t dc = (int64_t)d + sr->c;
  uint64_t ktail = dc < 0 ? 0 : (uint64_t)(dc / step) + 1u;
  uint64_t hend = k1 < ktail ? k1 : ktail;
  if (hend < k0) hend = k0;
  if (nthreads < 1) nthreads = 1;
  uint64_t hn = hend - k0;
  int nt = (uint64_t)nthreads > hn ? (int)(hn ? hn : 1) : nthreads;
  slice_job *jobs = (slice_job *)calloc((size_t)nt + 1, sizeof(slice_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
  for (int i = 0; i <= nt; ++i) {
    jobs[i].sr = *sr; jobs[i].step = step; jobs[i].alt = alt; jobs[i].d = d; jobs[i].P = P;
    jobs[i].acc = (uint32_t *)calloc(nw, sizeof(uint32_t));
  }
  for (int i = 0; i < nt; ++i) {
    jobs[i].k0 = k0 + hn * (uint64_t)i / (uint64_t)nt;
    jobs[i].k1 = k0 + hn * (uint64_t)(i + 1) / (uint64_t)nt;
  }
  jobs[nt].k0 = hend; jobs[nt].k1 = k1;          /* the tail part, if any */
  for (int i = 0; i < nt; ++i)
    if (nt > 1) pthread_create(&th[i], NULL, run_slice, &jobs[i]);
    else run_slice(&jobs[i]);
  if (nt > 1)
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  run_slice(&jobs[nt]);
  for (int i = 0; i <= nt; ++i) {
    add_mod(out, jobs[i].acc, nw, P);
    if (nterms) *nterms += jobs[i].nterms;
    free(jobs[i].acc);
  }
  free(jobs); free(th);
  return 0;
}

int pio_sum_slice(int formula, int j, uint64_t d, uint64_t k0, uint64_t k1, uint32_t P,
                  uint32_t *out, uint64_t *nterms, int nthreads) {
  pio_series tab[7];
  int32_t step, alt;
  int J = pio_series_table(formula, tab, &step, &alt);
  if (J < 0 || j < 0 || j >= J || P == 0 || k0 > k1) return -1;
  return sum_range(&tab[j], step, alt, d, k0, k1, P, out, nterms, nthreads);
}

/* Certification (section 3.1, adapted to truncation). Each summed term is
 * truncated by less than one unit of 2^-P, and the part of a series past its
 * stop index is below 2^-P/(1-2^-step) <= (16/15) 2^-P, so the exact
 * frac(2^d pi) lies within B = N + 2J units of S/2^P (modulo 1). With
 * G = S mod 2^(P-w), every number in that window has the same top w bits as S
 * exactly when G >= B and G + B <= 2^(P-w). */
int pio_certify(const uint32_t *S, uint32_t P, uint32_t w, uint64_t B) {
  uint32_t gb = P - w;                      /* guard bits */
  uint32_t nw = nwords(P) + 1;
  uint32_t *G = (uint32_t *)calloc(nw, sizeof(uint32_t));
  uint32_t *Bv = (uint32_t *)calloc(nw, sizeof(uint32_t));
  uint32_t *top = (uint32_t *)calloc(nw, sizeof(uint32_t));
  memcpy(G, S, sizeof(uint32_t) * nwords(P));
  clip(G, nw, gb);
  Bv[0] = (uint32_t)B; Bv[1] = (uint32_t)(B >> 32);
  /* G >= B ? */
  int ge = 1;
  for (uint32_t i = nw; i-- > 0;) {
    if (G[i] != Bv[i]) { ge = G[i] > Bv[i]; break; }
  }
  /* G + B <= 2^gb ?  i.e. 2^gb - G >= B */
  top[gb / 32] = 1u << (gb % 32);
  uint64_t borrow = 0;
  for (uint32_t i = 0; i < nw; ++i) {
    uint64_t dd = (uint64_t)top[i] - G[i] - borrow;
    top[i] = (uint32_t)dd;
    borrow = (dd >> 63) & 1u;
  }
  int le = 1;
  for (uint32_t i = nw; i-- > 0;) {
    if (top[i] != Bv[i]) { le = top[i] > Bv[i]; break; }
  }
  free(G); free(Bv); free(top);
  return ge && le;
}

int pio_extract(int formula, uint64_t n, uint32_t w, uint32_t P, uint32_t *S, uint64_t *N,
                int32_t *certified, int nthreads) {
  pio_series tab[7];
  int32_t step, alt;
  int J = pio_series_table(formula, tab, &step, &alt);
  if (J < 0 || n == 0 || w == 0 || P < w) return -1;
  uint64_t d = n - 1;            /* bit n after the radix point is the top bit of frac(2^(n-1) pi) */
  uint32_t nw = nwords(P);
  uint32_t *part = (uint32_t *)calloc(nw, sizeof(uint32_t));
  memset(S, 0, sizeof(uint32_t) * nw);
  uint64_t total = 0;
  for (int j = 0; j < J; ++j) {
    uint64_t cnt = 0;
    sum_range(&tab[j], step, alt, d, 0, UINT64_MAX, P, part, &cnt, nthreads);
    add_mod(S, part, nw, P);
    total += cnt;
  }
  free(part);
  if (N) *N = total;
  if (certified) *certified = pio_certify(S, P, w, total + 2u * (uint64_t)J);
  return 0;
}

/* ---- Machin's formula, for pinning ---------------------------------------- */

/* x = x / v (v < 2^32), returns nothing; x has nw words */
static void div_small(uint32_t *x, uint32_t nw, uint32_t v) {
  uint64_t rem = 0;
  for (uint32_t i = nw; i-- > 0;) {
    uint64_t cur = (rem << 32) | x[i];
    x[i] = (uint32_t)(cur / v);
    rem = cur % v;
  }
}

/* acc += or -= (16 or 4) * floor(2^F / x) series of atan(1/x):
 * atan(1/x) = sum_i (-1)^i / ((2i+1) x^(2i+1)). Returns the number of terms. */
static uint32_t atan_inv(uint32_t *acc, uint32_t nw, uint32_t F, uint32_t x, uint32_t mult,
                         int negate) {
  uint32_t *p = (uint32_t *)calloc(nw, sizeof(uint32_t));
  uint32_t *t = (uint32_t *)calloc(nw, sizeof(uint32_t));
  p[F / 32] = 1u << (F % 32);
  div_small(p, nw, x);                        /* p = 2^F / x */
  uint32_t i = 0;
  while (!is_zero(p, nw)) {
    memcpy(t, p, sizeof(uint32_t) * nw);
    div_small(t, nw, 2u * i + 1u);
    /* t *= mult */
    uint64_t carry = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      uint64_t v = (uint64_t)t[w] * mult + carry;
      t[w] = (uint32_t)v;
      carry = v >> 32;
    }
    int sub = (i & 1u) ^ (negate != 0);
    if (sub) sub_mod(acc, t, nw, 32u * nw);
    else add_mod(acc, t, nw, 32u * nw);
    div_small(p, nw, x * x);
    ++i;
  }
  free(p); free(t);
  return i;
}

int pio_machin(uint32_t nbits, uint32_t *out) {
  /* pi = 16 atan(1/5) - 4 atan(1/239) in fixed point with F = nbits + 64
   * fraction bits and two integer words of headroom */
  const uint32_t guard = 64;
  uint32_t F = nbits + guard;
  uint32_t nw = nwords(F) + 2;
  uint32_t *acc = (uint32_t *)calloc(nw, sizeof(uint32_t));
  uint32_t n1 = atan_inv(acc, nw, F, 5, 16, 0);
  uint32_t n2 = atan_inv(acc, nw, F, 239, 4, 1);
  /* p_i = floor(p_(i-1)/x^2) is low by less than 1 + 1/(x^2-1) units, and
   * t = floor(p_i/(2i+1)) by less than 3 units; times the multiplier, summed
   * over the terms, the value is off by at most errb units. */
  uint64_t errb = 3ull * 16u * (n1 + 1u) + 3ull * 4u * (n2 + 1u) + 64u;
  /* guard window = low 64 bits of acc */
  uint64_t g = (uint64_t)acc[0] | ((uint64_t)acc[1] << 32);
  int ok = g >= errb && g <= UINT64_MAX - errb;
  /* out = bits [guard, guard + nbits) of acc, i.e. the fraction bits of pi */
  uint32_t ow = nwords(nbits);
  for (uint32_t i = 0; i < ow; ++i) out[i] = acc[i + guard / 32];
  clip(out, ow, nbits);
  free(acc);
  return ok ? 0 : -1;
}
