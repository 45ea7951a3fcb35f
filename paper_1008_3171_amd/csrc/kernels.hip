// Kernels of the MI355X bit-extraction library.
//
//  head_kernel<L, ...>  the hot path: every head term (E >= 0, the A_k of
//                       eq (3.3)) of every series range it is given. A
//                       resident grid takes chunks of 256*run consecutive k
//                       of one series from a device counter; each lane owns
//                       run indices of one parity (so one sign) and sums its
//                       terms, and the workgroup folds the 256 lane sums into
//                       pending column sums that reach the query's
//                       carry-save counters with 2L atomics.
//  finalize_kernel<L>   one workgroup per query: the tail terms (the B_k of
//                       eq (3.3)) up to each series' stop index, the
//                       normalization of the carry-save counters, the
//                       certification of section 3.1 and the output limbs.
//
// The split of the index set into series ranges, chunks, waves and lanes is
// the multi-level partition of section 4 (jobs, tasks, threads) with the
// GPU's own levels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "arith.h"
#include "plan.h"

namespace pibbp {

// Series tables as (negative sign?, c, a, b): the series contributes
// sign * alt^k * 2^(d + c - step k) / (a k + b).
// Bellard, eq (1.2): +2^2/(10k+1) -1/(10k+3) -2^-4/(10k+5) -2^-4/(10k+7)
//                    +2^-6/(10k+9) -2^-1/(4k+1) -2^-6/(4k+3), times (-1)^k 2^-10k.
// BBP in the form of eq (3.1): +2^2/(8k+1) -2^-1/(2k+1) -1/(8k+5) -2^-1/(4k+3),
// times 2^-4k.
struct DevSeries {
  int32_t neg, c;
  uint32_t a, b;
};
__constant__ DevSeries kSeries[2][7] = {
    {{0, 2, 8, 1}, {1, -1, 2, 1}, {1, 0, 8, 5}, {1, -1, 4, 3}, {0, 0, 1, 1}, {0, 0, 1, 1}, {0, 0, 1, 1}},
    {{0, 2, 10, 1}, {1, 0, 10, 3}, {1, -4, 10, 5}, {1, -4, 10, 7}, {0, -6, 10, 9}, {1, -1, 4, 1},
     {1, -6, 4, 3}},
};
__constant__ int32_t kStep[2] = {4, 10};
__constant__ int32_t kAlt[2] = {0, 1};
__constant__ int32_t kNumSeries[2] = {4, 7};

// ---- one term --------------------------------------------------------------

// One term at L limbs by the R = 2^64 Montgomery ladder (any odd M < 2^60):
// t = floor(r 2^(64L) / M) with r = 2^E mod M, low bits below P cleared. The
// tail uses it with E = 0 for floor(2^(64L) / M). nb >= bit length of
// X = E + 64(L-1); extra leading zero bits only square the Montgomery one.
template <int L>
__device__ __forceinline__ void head_term64(uint64_t E, uint64_t M, uint32_t P, int nb,
                                            uint64_t (&t)[L]) {
  const uint64_t mp = neg_inv64(M);
  uint64_t x = mont_one64(M);
  const uint64_t X = E + 64ull * (L - 1);
  for (int j = nb - 1; j >= 0; --j) x = sqr_redc64(x, (uint32_t)(X >> j) & 1u, M, mp);
  x = x >= M ? x - M : x;  // s = 2^(E + 64L) mod M
  hensel64<L>(x, M, mp, t);
  clip_low<L>(t, P);
}

// ---- carry-save workgroup reduction -----------------------------------------

constexpr uint32_t kNoQuery = 0xffffffffu;

// Adds the 256 lane values v (L limbs each, mod 2^(64L)) to the workgroup's
// pending column sums. The lane values are first summed exactly: thread h adds
// up the 32-bit halves h of all lanes (below 2^40), then thread 0 propagates
// the carries, so each call adds one value below 2^32 to each pending column.
// (The 2L threads read one LDS bank at a time; a skewed start per thread
// would spread them over banks, but costs the head kernel 8 more VGPRs and a
// workgroup per CU, more than the fold's share of the time.) Pending columns belong to one query (counters at
// acc + pend_off, *pend_nc of them); a chunk of another query first flushes
// them into that query's carry-save counters with atomics. The counters stay
// exact while fewer than 2^32 chunks of one query are added up, which the
// host guarantees.
//
// Thread 0 also claims the workgroup's next chunk from the launch's counter
// (chunks 0 .. grid-1 are taken first, by block index); the fold's barriers
// publish it in *next. It is written after the first barrier, so every
// thread has read the previous value by then.
template <int L, int LMAX>
__device__ __forceinline__ void wg_fold(const uint64_t (&v)[L], uint32_t (*red)[256],
                                        unsigned long long *sums, unsigned long long *pend,
                                        uint32_t *pend_off, uint32_t *pend_nc, uint32_t acc_off,
                                        unsigned long long *acc, unsigned long long *ctr,
                                        unsigned long long *next) {
  const uint32_t tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    red[2 * i][tid] = (uint32_t)v[i];
    red[2 * i + 1][tid] = (uint32_t)(v[i] >> 32);
  }
  __syncthreads();
  if (tid < 2u * L) {
    unsigned long long s = 0;
    for (int i = 0; i < 256; ++i) s += red[tid][i];
    sums[tid] = s;
  }
  __syncthreads();
  if (tid == 0) {
    *next = gridDim.x + atomicAdd(ctr, 1ull);
    unsigned long long carry = 0;
    for (int h = 0; h < 2 * L; ++h) {
      const unsigned long long x = sums[h] + carry;
      sums[h] = x & 0xffffffffull;
      carry = x >> 32;
    }
  }
  __syncthreads();
  if (tid < 2u * LMAX) {
    const uint32_t cur = *pend_off;
    if (cur != acc_off) {
      if (cur != kNoQuery && tid < *pend_nc && pend[tid])
        atomicAdd(&acc[(uint64_t)cur + tid], pend[tid]);
      pend[tid] = 0;
    }
    if (tid < 2u * L) pend[tid] += sums[tid];
  }
  __syncthreads();
  if (tid == 0) {
    *pend_off = acc_off;
    *pend_nc = 2u * L;
  }
  __syncthreads();
}

// The workgroup's last flush of its pending column sums.
__device__ __forceinline__ void wg_flush(const unsigned long long *pend, const uint32_t *pend_off,
                                         const uint32_t *pend_nc, unsigned long long *acc) {
  const uint32_t tid = threadIdx.x;
  if (tid < *pend_nc && *pend_off != kNoQuery && pend[tid])
    atomicAdd(&acc[(uint64_t)*pend_off + tid], pend[tid]);
}

// ---- the head kernel ---------------------------------------------------------

// The first active lane's value of x, as a wave-uniform scalar. readfirstlane
// returns int: each half goes through uint32_t so it is not sign-extended.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ const HeadSeg &find_seg(const HeadSeg *segs, int nseg, uint64_t ch) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].chunk0 <= ch) lo = mid;
    else hi = mid - 1;
  }
  return segs[lo];
}

// Class-62 terms of one lane: k = k0, k0 + 2, ..., k0 + 2(run-1) (one
// parity, so one sign), accumulated unsigned into sum. M and the ladder
// exponent X = E + 64L - 62 step by 2a and -2 step.
//
// The ladder starts from an unreduced Montgomery one g = 2^62 - qM, with
// q = floor(2^62 / M_last) computed once for the run (M_last its largest
// modulus), so g == 2^62 (mod M) and 0 <= g < (e+1)M with
// e = floor(2^62/M) - q. Shifted left by the top `pre` exponent bits v, it is
// the Montgomery form of 2^v. The host sizes runs and `pre` so that
// (g 2^v)^2 < 2^60 M and g 2^v < 2^56, which keeps the first squaring inside
// its bounds; after it the residue is below 8M.
template <int L>
__device__ __forceinline__ void lane_run62(uint64_t k0, uint32_t run, uint32_t pre, uint64_t kend,
                                           uint64_t a, uint64_t b, uint64_t dc, uint64_t step,
                                           uint32_t P, uint64_t (&sum)[L]) {
  const uint64_t dM = 2u * a, ndX = 0u - 2u * uniform64(step);
  uint64_t M = a * k0 + b;
  uint64_t X = dc + 64ull * L - 62ull - step * k0;
  const uint32_t q = div_2_62(M + dM * (run - 1u));
  uint64_t msk[L];
  low_masks<L>(P, msk);
  // lane 0 holds the wave's smallest k, so the largest exponent: the wave
  // runs lane 0's term count nw, and lane 0's X bounds the ladder length
  const uint64_t ke = uniform64(kend), kw = uniform64(k0);
  const uint32_t nv = k0 < ke ? (uint32_t)((ke - k0 + 1u) >> 1) : 0u;
  const uint32_t nw = kw < ke ? min(run, (uint32_t)((ke - kw + 1u) >> 1)) : 0u;
  uint64_t Xw = uniform64(X);
  for (uint32_t i = 0; i < nw; ++i, M += dM, X += ndX, Xw += ndX) {
    const int nb0 = bitlen64(Xw);
    const uint32_t mp32 = neg_inv32((uint32_t)M);
    const uint32_t m0 = (uint32_t)M & kMask31, m1 = (uint32_t)(M >> 31);
    const uint32_t p = mp32 & kMask31;
    // the top t exponent bits v go into the start value: g 2^v == 2^(62+v)
    // is the Montgomery form of 2^v, so t squarings are skipped
    const int tb = pre < (uint32_t)nb0 ? (int)pre : nb0;
    const int nb = nb0 - tb;
    const uint32_t v = (uint32_t)(X >> nb) & ((1u << tb) - 1u);
    const uint64_t g = ((1ull << 62) - (uint64_t)q * M) << v;
    uint32_t d0 = (uint32_t)g & kMask31, d1 = (uint32_t)(g >> 31);
    const uint32_t xl = (uint32_t)X, xh = (uint32_t)(X >> 32);
    for (int j = nb - 33; j >= 0; --j) sqr_redc62(d0, d1, (xh >> j) & 1u, m0, m1, p);
    for (int j = (nb < 32 ? nb : 32) - 1; j >= 0; --j) sqr_redc62(d0, d1, (xl >> j) & 1u, m0, m1, p);
    uint64_t x = d0 + ((uint64_t)d1 << 31);  // == 2^(E + 64L) (mod M), below 8M
    x = x >= 4u * M ? x - 4u * M : x;
    x = x >= 2u * M ? x - 2u * M : x;
    x = x >= M ? x - M : x;
    uint64_t t[L];
    hensel_d32<L>(x, M, mp32, t);
    apply_masks<L>(t, msk);
    if (i < nv) add_limbs<L>(sum, t);
  }
}

// Binary64 terms of one lane, 2^29 <= M < 2^51: r = 2^E mod M by a
// left-to-right ladder over the bits of X = E in W-bit windows (W squarings, the
// window's value folded into the last one as a power of two); W = 4 for
// M < 2^33, 3 for M < 2^42, 2 for M < 2^48, and from there W = 5 with the
// window's value applied after its squarings as its own step (kSep). The top t = min(6, bitlen X) bits v of X
// give the start 2^v mod M directly; the remaining bits begin with one short
// window (their count mod W) and then whole windows at multiples of W. The
// whole windows above bit S = 32 - (32 mod W) are read from X >> S and the
// rest from the low word, so none straddles two words. The reciprocal of
// each modulus comes from the previous one by kNewton Newton steps (two
// below 2^33, where the moduli are closest together relatively). The term
// floor(r 2^P / M) is then divided out in binary64 digits (fp_term_digits),
// summed per digit position (with a carry step every kFpCarryTerms terms) and
// added to sum at the end of the run.
template <int L, int W, bool kSep, int kNewton>
__device__ __forceinline__ void lane_runf(uint64_t k0, uint32_t run, uint64_t kend, uint64_t a,
                                          uint64_t b, uint64_t dc, uint64_t step, uint32_t P,
                                          uint64_t (&sum)[L]) {
  constexpr int S = 32 - 32 % W;
  constexpr uint32_t kDigit = (1u << W) - 1u;
  constexpr int N = fp_digits(L), B = fp_digit_bits(L);
  const uint64_t dM = 2u * a, ndX = 0u - 2u * uniform64(step);
  uint64_t X = dc - step * k0;
  double Md = (double)(a * k0 + b);
  const double dMd = (double)dM;
  double inv = recip_f64(Md);
  int bits[N];
  fp_digit_sizes<N, B>(P, bits);
  double A[N];
#pragma unroll
  for (int d = 0; d < N; ++d) A[d] = 0.0;
  uint32_t nneg = 0;
  // terms of this lane inside the chunk (nv) and of lane 0 (nw: lane 0 has
  // the wave's smallest k, so the wave stops after nw terms); lane 0's
  // exponent, the wave's largest, is kept in scalar registers
  const uint64_t ke = uniform64(kend), kw = uniform64(k0);
  const uint32_t nv = k0 < ke ? (uint32_t)((ke - k0 + 1u) >> 1) : 0u;
  const uint32_t nw = kw < ke ? min(run, (uint32_t)((ke - kw + 1u) >> 1)) : 0u;
  uint64_t Xw = uniform64(X);
  for (uint32_t i0 = 0; i0 < nw; i0 += kFpCarryTerms) {
    const uint32_t i1 = min(nw, i0 + kFpCarryTerms);
    for (uint32_t i = i0; i < i1; ++i, X += ndX, Xw += ndX) {
      const int nb = bitlen64(Xw);
      const int rest = max(nb - 6, 0);
      const int lead = rest % W, top = rest - lead;
      double x = pow2_f64((uint32_t)(X >> rest), Md, inv);
      auto sq = [&](double y) { return sqr_f64(y, Md, inv); };
      auto sqd = [&](double y, uint32_t dg) {  // a window's last squaring and its digit
        return kSep ? scale_f64(sqr_f64(y, Md, inv), (int)dg, Md, inv)
                    : sqr_f64(y, (int)dg, Md, inv);
      };
      if (lead) {
        for (int j = 1; j < lead; ++j) x = sq(x);
        x = sqd(x, (uint32_t)(X >> top) & ((1u << lead) - 1u));
      }
      const uint32_t xhi = (uint32_t)(X >> S), xlo = (uint32_t)X;
      for (int p = top - W; p >= S; p -= W) {
#pragma unroll
        for (int j = 1; j < W; ++j) x = sq(x);
        x = sqd(x, (xhi >> (p - S)) & kDigit);
      }
      for (int p = (top < S ? top : S) - W; p >= 0; p -= W) {
#pragma unroll
        for (int j = 1; j < W; ++j) x = sq(x);
        x = sqd(x, (xlo >> p) & kDigit);
      }
      // x == 2^E (mod M), |x| < M; lanes past the chunk's end sit this out
      if (i < nv) fp_term_digits<N>(x, Md, inv, bits, A, nneg);
      Md += dMd;
      inv = recip_step(Md, inv);
      if (kNewton > 1) inv = recip_step(Md, inv);
    }
    fp_carry_digits<N, B>(A, nneg);
  }
  fp_digits_to_limbs<L>(A, nneg, P, sum);
}

// Class-32 terms of one lane (R = 2^32; X = E + 64L - 32). Below 2^29 the
// residues stay in [0, 2M): a Montgomery squaring is 3 instructions, and W-bit
// exponent windows (W = 3 below 2^23, 2 below 2^27, else 1) apply each
// window's digit as 2^d in its last squaring (2 more). With kReduced
// (2^29 <= M < 2^31, one-bit windows) every squaring result is brought below
// M (2 more): from x < M, x (x << b) < 2M^2 and the REDC result is below 2M. The bits of X start
// with one short window (bitlen mod W bits); whole windows above bit
// S = 32 - (32 mod W) are read from X >> S. Two start values:
//  * kRunStart (M >= 2^22): the Montgomery one is g = 2^32 - qM with
//    q = floor(2^32 / M_last) for the lane's run; the host keeps runs short
//    enough that g < 2M. Below 2^22 it comes from doublings of 2^bl - M.
// The k = 0 term of a b = 1 series has M = 1 and value 2^E mod 1 = 0; it is
// computed on garbage and not added.
template <int L, int W, bool kRunStart, bool kReduced = false>
__device__ __forceinline__ void lane_run32(uint64_t k0, uint32_t run, uint64_t kend, uint64_t a,
                                           uint64_t b, uint64_t dc, uint64_t step, uint32_t P,
                                           uint64_t (&sum)[L]) {
  constexpr int S = 32 - 32 % W;
  constexpr uint32_t kDigit = (1u << W) - 1u;
  const uint64_t dM = 2u * a, ndX = 0u - 2u * uniform64(step);
  uint64_t M = a * k0 + b;
  uint64_t X = dc + 64ull * L - 32ull - step * k0;
  uint32_t q = 0;
  if (kRunStart) q = div_2_32((uint32_t)(M + dM * (run - 1u)));
  uint64_t msk[L];
  low_masks<L>(P, msk);
  const uint64_t ke = uniform64(kend), kw = uniform64(k0);
  const uint32_t nv = k0 < ke ? (uint32_t)((ke - k0 + 1u) >> 1) : 0u;
  const uint32_t nw = kw < ke ? min(run, (uint32_t)((ke - kw + 1u) >> 1)) : 0u;
  uint64_t Xw = uniform64(X);
  for (uint32_t i = 0; i < nw; ++i, M += dM, X += ndX, Xw += ndX) {
    const int nb = bitlen64(Xw);
    const int lead = nb % W, top = nb - lead;
    const uint32_t M32 = (uint32_t)M;
    const uint32_t mp = neg_inv32(M32);
    uint32_t x = kRunStart ? 0u - q * M32 : mont_one32(M32);  // below 2M
    if (kReduced) x = min(x, x - M32);
    if (lead) {
      for (int j = 1; j < lead; ++j) x = sqr_redc32_plain(x, M32, mp);
      x = sqr_redc32_digit(x, (uint32_t)(X >> top) & ((1u << lead) - 1u), M32, mp);
    }
    const uint32_t xhi = (uint32_t)(X >> S), xlo = (uint32_t)X;
    for (int p = top - W; p >= S; p -= W) {
#pragma unroll
      for (int j = 1; j < W; ++j) x = sqr_redc32_plain(x, M32, mp);
      x = sqr_redc32_digit(x, (xhi >> (p - S)) & kDigit, M32, mp);
      if (kReduced) x = min(x, x - M32);
    }
    for (int p = (top < S ? top : S) - W; p >= 0; p -= W) {
#pragma unroll
      for (int j = 1; j < W; ++j) x = sqr_redc32_plain(x, M32, mp);
      x = sqr_redc32_digit(x, (xlo >> p) & kDigit, M32, mp);
      if (kReduced) x = min(x, x - M32);
    }
    x = min(x, x - M32);
    uint64_t t[L];
    hensel32<L>(x, M32, mp, t);
    apply_masks<L>(t, msk);
    if (i < nv && M32 != 1u) add_limbs<L>(sum, t);
  }
}

// The limb count a query of P bits runs at: the smallest instantiated kernel
// limb class holding P (1-6, 8, 12 or 17 limbs).
__device__ __forceinline__ int limb_class_of(uint32_t P) {
  const int Lq = (int)((P + 63u) / 64u);
  return Lq <= 6 ? Lq : Lq <= 8 ? 8 : Lq <= 12 ? 12 : 17;
}

// One chunk of one segment at L limbs: every lane sums its run of terms, the
// sum takes the lanes' common sign, and the workgroup folds the lane sums.
template <int L, int LMAX>
__device__ __forceinline__ void head_chunk(const HeadSeg &sg, uint64_t ch, uint32_t (*red)[256],
                                           unsigned long long *sums, unsigned long long *pend,
                                           uint32_t *pend_off, uint32_t *pend_nc,
                                           unsigned long long *acc, unsigned long long *ctr,
                                           unsigned long long *next) {
  const uint32_t tid = threadIdx.x;
  const uint32_t pair = tid >> 1, par = tid & 1u;
  const uint32_t run = sg.run;
  const uint64_t CH = 256ull * run;
  const uint64_t kc = sg.kb + (ch - sg.chunk0) * CH;
  const uint64_t kend = kc + CH < sg.ke ? kc + CH : sg.ke;
  const DevSeries sr = kSeries[sg.formula][sg.j];
  const uint64_t step = (uint64_t)kStep[sg.formula];
  const uint64_t k0 = kc + 2ull * run * pair + par;
  // every k of this lane has the parity of k0, so one sign for the chunk
  const bool neg = (sr.neg != 0) ^ (kAlt[sg.formula] != 0 && (k0 & 1u));
  const uint64_t dc = sg.d + (uint64_t)(int64_t)sr.c;
  uint64_t sum[L];
#pragma unroll
  for (int i = 0; i < L; ++i) sum[i] = 0;
  switch (sg.cls) {
    case 64: lane_run62<L>(k0, run, sg.pre, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 51: lane_runf<L, 5, true, 1>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 48: lane_runf<L, 2, false, 1>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 42: lane_runf<L, 3, false, 1>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 33: lane_runf<L, 4, false, 2>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 31: lane_run32<L, 1, true, true>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 29: lane_run32<L, 1, true>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    case 27: lane_run32<L, 2, true>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
    default: lane_run32<L, 3, false>(k0, run, kend, sr.a, sr.b, dc, step, sg.P, sum); break;
  }
  if (neg) neg_limbs<L>(sum);
  wg_fold<L, LMAX>(sum, red, sums, pend, pend_off, pend_nc, sg.acc_off, acc, ctr, next);
}

// Chunks are handed out dynamically: each workgroup starts at its block
// index and then takes the next unclaimed chunk from *ctr (zero at launch),
// so workgroups that draw cheap chunks keep working until the last one.
// An instance serves queries of LLO to LHI limbs: one limb count (the single
// query, and batches of 8, 12 or 17 limbs) or every count from 1 to 6 in one
// launch (batches and serving steps), each chunk run at its query's count.
template <int LLO, int LHI>
__device__ void head_chunks(const HeadSeg *segs, int nseg, uint64_t nchunks,
                            unsigned long long *acc, unsigned long long *ctr) {
  __shared__ uint32_t red[2 * LHI][256];
  __shared__ unsigned long long sums[2 * LHI], pend[2 * LHI], next;
  __shared__ uint32_t pend_off, pend_nc;
  const uint32_t tid = threadIdx.x;
  if (tid < 2u * LHI) pend[tid] = 0;
  if (tid == 0) {
    pend_off = kNoQuery;
    pend_nc = 0;
  }
  __syncthreads();
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch = next) {
    const HeadSeg sg = find_seg(segs, nseg, ch);
#define PIBBP_CHUNK(L) head_chunk<L, LHI>(sg, ch, red, sums, pend, &pend_off, &pend_nc, acc, ctr, &next)
    if constexpr (LLO == LHI) {
      PIBBP_CHUNK(LHI);
    } else {
      static_assert(LLO == 1 && LHI == 6, "fused instances cover 1 to 6 limbs");
      switch (limb_class_of(sg.P)) {
        case 1: PIBBP_CHUNK(1); break;
        case 2: PIBBP_CHUNK(2); break;
        case 3: PIBBP_CHUNK(3); break;
        case 4: PIBBP_CHUNK(4); break;
        case 5: PIBBP_CHUNK(5); break;
        default: PIBBP_CHUNK(6); break;
      }
    }
#undef PIBBP_CHUNK
  }
  wg_flush(pend, &pend_off, &pend_nc, acc);
}

template <int L>
__global__ __launch_bounds__(256) void head_kernel_args(HeadSegTable tab, uint64_t nchunks,
                                                        unsigned long long *acc,
                                                        unsigned long long *ctr) {
  head_chunks<L, L>(tab.s, tab.n, nchunks, acc, ctr);
}

template <int L>
__global__ __launch_bounds__(256) void head_kernel_ptr(const HeadSeg *segs, int nseg,
                                                       uint64_t nchunks, unsigned long long *acc,
                                                       unsigned long long *ctr) {
  head_chunks<L, L>(segs, nseg, nchunks, acc, ctr);
}

// Every query of 1 to 6 limbs in one persistent launch. Held to 80 VGPRs (six
// waves per SIMD, as the one-count pointer instances), which it meets without
// spilling; unbounded it takes 96 and runs five.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void head_kernel_fused(const HeadSeg *segs, int nseg,
                                                         uint64_t nchunks, unsigned long long *acc,
                                                         unsigned long long *ctr) {
  head_chunks<1, 6>(segs, nseg, nchunks, acc, ctr);
}

__global__ void zero_kernel(unsigned long long *p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---- tail terms and finalize ------------------------------------------------

// Tail term (E < 0) at L limbs: floor(2^(64L+E) / M) with its low 64L - P bits
// cleared.
// For M > 1 it is floor(2^(64L)/M) shifted right by -E (the same floor), and
// floor(2^(64L)/M) is the head formula with E = 0 (r = 1).
template <int L>
__device__ void tail_term(int64_t E, uint64_t M, uint32_t P, uint64_t (&t)[L]) {
  const int64_t e = 64ll * L + E;
#pragma unroll
  for (int i = 0; i < L; ++i) t[i] = 0;
  if (e < 0) return;
  if (M == 1) {
    const int li = (int)(e >> 6);
#pragma unroll
    for (int i = 0; i < L; ++i)
      if (i == li) t[i] = 1ull << (e & 63);
  } else {
    uint64_t full[L];
    head_term64<L>(0, M, 64u * L, bitlen64(64ull * (L - 1)), full);
    const int sh = (int)(-E);
    const int ls = sh >> 6, bs = sh & 63;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      uint64_t lo = 0, hi = 0;
#pragma unroll
      for (int s = 0; s < L; ++s) {
        if (s == i + ls) lo = full[s];
        if (s == i + ls + 1) hi = full[s];
      }
      t[i] = bs ? (lo >> bs) | (hi << (64 - bs)) : lo;
    }
  }
  clip_low<L>(t, P);
}

// Certification (section 3.1, adapted to truncated terms). S is given in
// Lq left-aligned limbs (z = 64Lq - P zero bits at the bottom). G = the low
// g = 64Lq - w bits, B = (N + 2J) 2^z; the top w bits are proven bits of pi
// iff G >= B and G + B <= 2^g. Both tests run over Lq + 1 limbs.
// mode 1: certify; mode 2: report N only (code PI_OK), for slices.
__device__ pi_status certify(const uint64_t *Sq, int Lq, uint32_t P, uint32_t w, uint64_t N,
                             uint64_t J, uint32_t mode) {
  pi_status st;
  st.reserved = 0;
  st.nterms = N;
  if (mode == 2) {
    st.code = PI_OK;
    return st;
  }
  const uint32_t z = 64u * (uint32_t)Lq - P, g = 64u * (uint32_t)Lq - w;
  const uint64_t Bn = N + 2ull * J;
  uint64_t Bv[PI_MAX_L + 1], Gv[PI_MAX_L + 1], Sum[PI_MAX_L + 1], Pg[PI_MAX_L + 1];
  for (int i = 0; i <= Lq; ++i) {
    Bv[i] = 0;
    Pg[i] = 0;
    const uint32_t lo = 64u * (uint32_t)i;
    uint64_t gi = 0;
    if (i < Lq) gi = g >= lo + 64u ? Sq[i] : (g > lo ? Sq[i] & ((1ull << (g - lo)) - 1ull) : 0ull);
    Gv[i] = gi;
    if (g >= lo && g < lo + 64u) Pg[i] = 1ull << (g - lo);
  }
  Bv[0] = Bn << z;
  if (z) Bv[1] = Bn >> (64u - z);
  unsigned long long c1 = 0, c2 = 0, c3 = 0;
  for (int i = 0; i <= Lq; ++i) {
    (void)__builtin_subcll(Gv[i], Bv[i], c1, &c1);      // G - B: borrow out => G < B
    Sum[i] = __builtin_addcll(Gv[i], Bv[i], c2, &c2);  // G + B
  }
  for (int i = 0; i <= Lq; ++i) (void)__builtin_subcll(Pg[i], Sum[i], c3, &c3);  // 2^g - (G+B)
  st.code = (c1 == 0 && c2 == 0 && c3 == 0) ? PI_OK : PI_UNCERTAIN;
  return st;
}

// Sum of `count` partial sums (each Lq left-aligned limbs, mod 2^(64Lq)) and
// the certification of the total with N = nterms: the final sum over jobs of
// section 4, for sums kept outside the device between calls. One workgroup.
__global__ __launch_bounds__(256) void combine_kernel(const uint64_t *parts, int count, int Lq,
                                                     uint32_t P, uint32_t w, uint64_t nterms,
                                                     uint32_t J, uint64_t *out, pi_status *status) {
  __shared__ unsigned long long col[2 * PI_MAX_L];
  const uint32_t tid = threadIdx.x;
  if (tid < 2u * PI_MAX_L) col[tid] = 0;
  __syncthreads();
  // carry-save: every 32-bit half of every part goes into its column
  for (int i = tid; i < count * 2 * Lq; i += 256) {
    const int part = i / (2 * Lq), h = i % (2 * Lq);
    const uint64_t limb = parts[(uint64_t)part * Lq + h / 2];
    atomicAdd(&col[h], (unsigned long long)(uint32_t)(h & 1 ? limb >> 32 : limb));
  }
  __syncthreads();
  if (tid != 0) return;
  uint64_t S[PI_MAX_L];
  unsigned long long carry = 0;
  for (int i = 0; i < Lq; ++i) {
    const unsigned long long lo = col[2 * i] + carry;
    carry = (lo >> 32) + (lo < carry ? (1ull << 32) : 0ull);
    const unsigned long long hi = col[2 * i + 1] + carry;
    carry = (hi >> 32) + (hi < carry ? (1ull << 32) : 0ull);
    S[i] = (lo & 0xffffffffull) | (hi << 32);
  }
  for (int i = 0; i < Lq; ++i) out[i] = S[i];
  if (status) *status = certify(S, Lq, P, w, nterms, J, 1);
}

// One query's finalization at L limbs (one workgroup; LDS sized for LMAX).
template <int L, int LMAX>
__device__ void finalize_query(const FinQuery &q, const unsigned long long *acc, uint64_t *out,
                               pi_status *status, uint32_t (*red)[256], unsigned long long *cnt,
                               unsigned long long &nz_total) {
  const uint32_t tid = threadIdx.x;
  const int f = (int)q.formula;
  const int J = kNumSeries[f];
  const int64_t step = kStep[f];
  if (tid == 0) nz_total = 0;
  uint64_t ntail = 0;
  for (int j = 0; j < J; ++j) ntail += q.tk1[j] - q.tk0[j];
  uint64_t sum[L];
#pragma unroll
  for (int i = 0; i < L; ++i) sum[i] = 0;
  unsigned long long nz = 0;
  // tail items of all series, flattened; a few hundred at most
  for (uint64_t it = tid; it < ntail; it += 256) {
    uint64_t r = it;
    int j = 0;
    while (r >= q.tk1[j] - q.tk0[j]) {
      r -= q.tk1[j] - q.tk0[j];
      ++j;
    }
    const uint64_t k = q.tk0[j] + r;
    const DevSeries sr = kSeries[f][j];
    const int64_t E = (int64_t)q.d + sr.c - step * (int64_t)k;
    const uint64_t M = (uint64_t)sr.a * k + sr.b;
    uint64_t t[L];
    tail_term<L>(E, M, q.P, t);
    bool nonzero = false;
#pragma unroll
    for (int i = 0; i < L; ++i) nonzero |= t[i] != 0;
    nz += nonzero ? 1u : 0u;
    const bool neg = (sr.neg != 0) ^ (kAlt[f] != 0 && (k & 1u));
    if (neg) neg_limbs<L>(t);
    add_limbs<L>(sum, t);
  }
  if (tid < 2u * L) cnt[tid] = acc[(uint64_t)q.acc_off + tid];
  __syncthreads();
  if (nz) atomicAdd(&nz_total, nz);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    red[2 * i][tid] = (uint32_t)sum[i];
    red[2 * i + 1][tid] = (uint32_t)(sum[i] >> 32);
  }
  __syncthreads();
  if (tid < 2u * L) {
    unsigned long long s = cnt[tid];
    for (int i = 0; i < 256; ++i) s += red[tid][i];
    cnt[tid] = s;
  }
  __syncthreads();
  if (tid != 0) return;
  // normalize the carry-save counters: S = sum_h cnt[h] 2^(32h) mod 2^(64L)
  uint64_t S[PI_MAX_L];
  unsigned long long carry = 0;
  for (int i = 0; i < L; ++i) {
    const unsigned long long lo = cnt[2 * i] + carry;
    carry = (lo >> 32) + (lo < carry ? (1ull << 32) : 0ull);
    const unsigned long long hi = cnt[2 * i + 1] + carry;
    carry = (hi >> 32) + (hi < carry ? (1ull << 32) : 0ull);
    S[i] = (lo & 0xffffffffull) | (hi << 32);
  }
  // the query's result is the top Lq limbs (the lower L - Lq are zero)
  const int Lq = (int)q.Lq;
  const uint64_t *Sq = S + (L - Lq);
  uint64_t *o = out + q.out_off;
  for (int i = 0; i < Lq; ++i) o[i] = Sq[i];
  if (!q.want_status) return;
  status[q.status_idx] = certify(Sq, Lq, q.P, q.w, q.nhead + nz_total, (uint64_t)J,
                                  q.want_status);
}

template <int L>
__global__ __launch_bounds__(256) void finalize_kernel(FinQuery single, const FinQuery *qs,
                                                       const unsigned long long *acc,
                                                       uint64_t *out, pi_status *status) {
  __shared__ uint32_t red[2 * L][256];
  __shared__ unsigned long long cnt[2 * L];
  __shared__ unsigned long long nz_total;
  const FinQuery q = qs ? qs[blockIdx.x] : single;
  finalize_query<L, L>(q, acc, out, status, red, cnt, nz_total);
}

// Queries of 1 to 6 limbs in one launch, a workgroup each at its own count.
__global__ __launch_bounds__(256) void finalize_kernel_fused(const FinQuery *qs,
                                                             const unsigned long long *acc,
                                                             uint64_t *out, pi_status *status) {
  __shared__ uint32_t red[12][256];
  __shared__ unsigned long long cnt[12];
  __shared__ unsigned long long nz_total;
  const FinQuery q = qs[blockIdx.x];
  switch (limb_class_of(q.P)) {
    case 1: finalize_query<1, 6>(q, acc, out, status, red, cnt, nz_total); break;
    case 2: finalize_query<2, 6>(q, acc, out, status, red, cnt, nz_total); break;
    case 3: finalize_query<3, 6>(q, acc, out, status, red, cnt, nz_total); break;
    case 4: finalize_query<4, 6>(q, acc, out, status, red, cnt, nz_total); break;
    case 5: finalize_query<5, 6>(q, acc, out, status, red, cnt, nz_total); break;
    default: finalize_query<6, 6>(q, acc, out, status, red, cnt, nz_total); break;
  }
}

// ---- launchers ---------------------------------------------------------------

template <int L>
static hipError_t launch_head_args_L(const HeadSegTable &tab, uint64_t nchunks, int grid,
                                     unsigned long long *acc, unsigned long long *ctr,
                                     hipStream_t st) {
  hipLaunchKernelGGL(head_kernel_args<L>, dim3(grid), dim3(256), 0, st, tab, nchunks, acc, ctr);
  return hipGetLastError();
}
template <int L>
static hipError_t launch_head_ptr_L(const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                                    unsigned long long *acc, unsigned long long *ctr,
                                    hipStream_t st) {
  hipLaunchKernelGGL(head_kernel_ptr<L>, dim3(grid), dim3(256), 0, st, segs, nseg, nchunks, acc,
                     ctr);
  return hipGetLastError();
}
template <int L>
static hipError_t launch_fin_L(const FinQuery &single, const FinQuery *qs, int nq,
                               const unsigned long long *acc, uint64_t *out, pi_status *status,
                               hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel<L>, dim3(nq), dim3(256), 0, st, single, qs, acc, out, status);
  return hipGetLastError();
}

hipError_t launch_head_fused(const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                            unsigned long long *acc, unsigned long long *ctr, hipStream_t st) {
  hipLaunchKernelGGL(head_kernel_fused, dim3(grid), dim3(256), 0, st, segs, nseg, nchunks, acc,
                     ctr);
  return hipGetLastError();
}

hipError_t launch_finalize_fused(const FinQuery *qs, int nq, const unsigned long long *acc,
                                 uint64_t *out, pi_status *status, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel_fused, dim3(nq), dim3(256), 0, st, qs, acc, out, status);
  return hipGetLastError();
}

int head_occupancy_fused() {
  int n = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, head_kernel_fused, 256, 0) == hipSuccess
             ? n
             : 0;
}

#define PIBBP_DISPATCH(Lk, CALL)                     \
  switch (Lk) {                                      \
    case 1: return CALL(1);                          \
    case 2: return CALL(2);                          \
    case 3: return CALL(3);                          \
    case 4: return CALL(4);                          \
    case 5: return CALL(5);                          \
    case 6: return CALL(6);                          \
    case 8: return CALL(8);                          \
    case 12: return CALL(12);                        \
    case 17: return CALL(17);                        \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_head_args(int Lk, const HeadSegTable &tab, uint64_t nchunks, int grid,
                            unsigned long long *acc, unsigned long long *ctr, hipStream_t st) {
#define C(L) launch_head_args_L<L>(tab, nchunks, grid, acc, ctr, st)
  PIBBP_DISPATCH(Lk, C)
#undef C
}
hipError_t launch_head_ptr(int Lk, const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                           unsigned long long *acc, unsigned long long *ctr, hipStream_t st) {
#define C(L) launch_head_ptr_L<L>(segs, nseg, nchunks, grid, acc, ctr, st)
  PIBBP_DISPATCH(Lk, C)
#undef C
}
hipError_t launch_finalize(int Lk, const FinQuery &single, const FinQuery *qs, int nq,
                           const unsigned long long *acc, uint64_t *out, pi_status *status,
                           hipStream_t st) {
#define C(L) launch_fin_L<L>(single, qs, nq, acc, out, status, st)
  PIBBP_DISPATCH(Lk, C)
#undef C
}
hipError_t launch_combine(const uint64_t *parts, int count, int Lq, uint32_t P, uint32_t w,
                          uint64_t nterms, uint32_t J, uint64_t *out, pi_status *status,
                          hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(256), 0, st, parts, count, Lq, P, w, nterms, J,
                     out, status);
  return hipGetLastError();
}

template <int L>
static int occupancy_L(bool by_value) {
  int n = 0;
  const hipError_t e =
      by_value ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, head_kernel_args<L>, 256, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, head_kernel_ptr<L>, 256, 0);
  return e == hipSuccess ? n : 0;
}

int head_occupancy(int Lk, bool by_value) {
#define C(L) occupancy_L<L>(by_value)
  switch (Lk) {
    case 1: return C(1);
    case 2: return C(2);
    case 3: return C(3);
    case 4: return C(4);
    case 5: return C(5);
    case 6: return C(6);
    case 8: return C(8);
    case 12: return C(12);
    case 17: return C(17);
    default: return 0;
  }
#undef C
}

// ---- static scratch ---------------------------------------------------------

// The scratch of pi_extract_noalloc, for callers that cannot allocate: one
// query's 2L carry-save counters and its head launch's chunk counter (at most
// 2 * 17 + 1 words). Each device holds its own copy until the process ends,
// and every such call on a device shares it.
constexpr uint32_t kStaticScratchWords = 64;
static __device__ __align__(256) unsigned long long scratch[kStaticScratchWords];

// In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from the runtime, once per device, with that device
// current, and only that address is ever passed to a kernel.
constexpr int kMaxDevices = 64;

hipError_t static_scratch(unsigned long long **ptr, uint32_t *words) {
  static std::mutex mu;
  static unsigned long long *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = (unsigned long long *)p;
  }
  *ptr = addr[dev];
  *words = kStaticScratchWords;
  return hipSuccess;
}

hipError_t launch_zero(unsigned long long *p, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace pibbp
