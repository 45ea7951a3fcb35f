/* CPU model of the head kernel's binary64 modular squaring, for checking its
 * exactness bounds (test infrastructure; not part of the library).
 *
 * A residue is an integer-valued double |x| < M. One step forms
 * y = 2^d x^2 - qM as the kernel does: H = x * (2^d x) rounded,
 * Lo = fma(x, 2^d x, -H), q = rint(H * inv), y = fma(-q, M, H) + Lo, and for
 * moduli from 2^48 a second reduction y - rint(y * inv) M after each window.
 *
 * Reads lines "M d x re inv_mode" on stdin (inv_mode 0: inv = 1/M correctly
 * rounded; 1: one Newton step from 1/(M - 20), as after the previous modulus
 * of a lane with a = 10; 2: two such steps) and prints "y ok" per line,
 * where ok is 1 when both intermediate results were below 2^53 in magnitude
 * (so exact) and |y| < M.
 * "W M W d x re inv_mode" lines run one W-bit window with digit d from x and
 * print "y ok" (ok: every intermediate below 2^53). re 0: the digit goes into
 * the window's last squaring; 1: the same, then a second reduction; 2: W
 * plain squarings, then the digit applied on its own as 2^d y reduced by one
 * rounded quotient. "L M X W re steps" lines print the full ladder's
 * 2^X mod M (steps: Newton steps per modulus, as in inv_mode).
 * "D M x P B N inv_mode" lines divide x 2^P by M in N signed digits, most
 * significant first: ne = ceil(P / B) digits of B bits, the top one holding
 * P - (ne - 1)B, and 0-bit digits above it. Each digit is
 * q = fma(y 2^b, inv, 1.5 * 2^52) - 1.5 * 2^52, y <- fma(-q, M, y 2^b). Prints
 * the N digits from the top, then 1 if the last remainder is negative, then
 * ok (every remainder below M in magnitude and every rounded product below
 * 2^51, so every step exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static double newton(double m, double r) {
  const double e = fma(-m, r, 1.0);
  return fma(r, e, r);
}

static double inverse(double M, int mode) {
  if (mode == 0) return 1.0 / M;
  const double r = newton(M, 1.0 / (M - 20.0));
  return mode == 1 ? r : newton(M, r);
}

/* re 0: ok also needs |y| < M; re 1: a second reduction follows; re 2:
 * only exactness is asked (the result may exceed M). */
static int step(double x, int d, double M, double inv, int re, double *out) {
  const double xs = ldexp(x, d);
  const double h = x * xs;
  const double lo = fma(x, xs, -h);
  const double q = rint(h * inv);
  const double r0 = fma(-q, M, h);
  double y = r0 + lo;
  int ok = fabs(r0) < 0x1p53 && fabs(y) < 0x1p53;
  if (re == 1) y = fma(-rint(y * inv), M, y);
  *out = y;
  return ok && (re || fabs(y) < M);
}

/* The digit applied on its own: y = 2^d x - rint(2^d x * inv) M. ok when the
 * quotient is an exact integer (below 2^52) and the result is exact. */
static int scale(double x, int d, double M, double inv, double *out) {
  const double xs = ldexp(x, d);
  const double q = rint(xs * inv);
  const double y = fma(-q, M, xs);
  *out = y;
  return fabs(q) < 0x1p52 && fabs(y) < 0x1p53;
}

/* One W-bit window. re 0: W - 1 plain squarings and one with the digit d;
 * re 1: the same, then a second reduction; re 2: W plain squarings, then the
 * digit applied on its own (scale). ok when every intermediate stayed exact. */
static int window(double x, int W, int d, double M, double inv, int re, double *out) {
  if (re == 2) {
    for (int j = 0; j < W; ++j)
      if (!step(x, 0, M, inv, 2, &x)) return 0;
    return scale(x, d, M, inv, out);
  }
  for (int j = 1; j < W; ++j)
    if (!step(x, 0, M, inv, 0, &x)) return 0;
  return step(x, d, M, inv, re, out);
}

/* 2^X mod M by the kernel's ladder: start 2^v for the top 6 bits, one short
 * window, then W-bit windows; returns the residue in [0, M) or -1. */
static long long ladder(unsigned long long M, unsigned long long X, int W, int re, int steps) {
  const double Md = (double)M, inv = inverse(Md, steps);
  const int nb = X ? 64 - __builtin_clzll(X) : 0;
  const int rest = nb < 6 ? 0 : nb - 6;
  const int lead = rest % W, top = rest - lead;
  const double p = ldexp(1.0, (int)(X >> rest));
  double x = fma(-rint(p * inv), Md, p);
  if (fabs(x) >= Md) return -1;
  if (lead && !window(x, lead, (int)((X >> top) & ((1u << lead) - 1u)), Md, inv, re, &x))
    return -1;
  for (int q = top - W; q >= 0; q -= W)
    if (!window(x, W, (int)((X >> q) & ((1u << W) - 1u)), Md, inv, re, &x)) return -1;
  x = fma(-floor(x * inv), Md, x);  /* [0, M): x * inv stays inside (-1, 1) */
  if (x < 0 || x >= Md) return -1;
  double y = x + 0x1p52;
  unsigned long long u;
  memcpy(&u, &y, 8);
  return (long long)(u & ((1ull << 52) - 1u));
}

int main(void) {
  char kind[8];
  while (scanf("%7s", kind) == 1) {
    if (kind[0] == 'D') {
      double M, x;
      int P, B, N, mode;
      if (scanf("%lf %lf %d %d %d %d", &M, &x, &P, &B, &N, &mode) != 6) return 1;
      const double inv = inverse(M, mode), C = 0x1.8p52;
      const int ne = (P + B - 1) / B, bt = P - (ne - 1) * B;
      double y = x;
      int ok = fabs(x) < M;
      for (int d = N - 1; d >= 0; --d) {
        const int b = d < ne - 1 ? B : d == ne - 1 ? bt : 0;
        const double ys = ldexp(y, b);
        ok = ok && fabs(ys * inv) < 0x1p51;
        const double q = fma(ys, inv, C) - C;
        y = fma(-q, M, ys);
        ok = ok && fabs(y) < M;
        printf("%.0f ", q);
      }
      printf("%d %d\n", y < 0.0, ok);
    } else if (kind[0] == 'W') {
      double M, x;
      int W, d, re, mode;
      if (scanf("%lf %d %d %lf %d %d", &M, &W, &d, &x, &re, &mode) != 6) return 1;
      double y;
      const int ok = window(x, W, d, M, inverse(M, mode), re, &y);
      printf("%.0f %d\n", y, ok);
    } else if (kind[0] == 'S') {
      double M, x;
      int d, re, mode;
      if (scanf("%lf %d %lf %d %d", &M, &d, &x, &re, &mode) != 5) return 1;
      double y;
      const int ok = step(x, d, M, inverse(M, mode), re, &y);
      printf("%.0f %d\n", y, ok);
    } else {
      unsigned long long M, X;
      int W, re, steps;
      if (scanf("%llu %llu %d %d %d", &M, &X, &W, &re, &steps) != 5) return 1;
      printf("%lld\n", ladder(M, X, W, re, steps));
    }
  }
  return 0;
}
