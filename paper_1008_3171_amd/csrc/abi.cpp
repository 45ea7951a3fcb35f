// C ABI of the library: argument checks, the host-side partition of each
// query's index set, scratch memory, and kernel launches.
//
// The partition follows section 4's multi-level split (the final sum over
// jobs, each over tasks, each over threads): a query's index set is split by
// series j and by modulus class into head segments, each segment into chunks
// of 256*run consecutive indices (one workgroup pass), each chunk into lanes.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "host.h"
#include "pibbp.h"
#include "plan.h"

namespace pibbp {
namespace host {

struct HostSeries {
  int neg, c;
  uint64_t a, b;
};
// Same data as the device tables: eq (1.2) for Bellard, eq (3.1) for BBP.
const HostSeries kHSeries[2][7] = {
    {{0, 2, 8, 1}, {1, -1, 2, 1}, {1, 0, 8, 5}, {1, -1, 4, 3}, {0, 0, 1, 1}, {0, 0, 1, 1}, {0, 0, 1, 1}},
    {{0, 2, 10, 1}, {1, 0, 10, 3}, {1, -4, 10, 5}, {1, -4, 10, 7}, {0, -6, 10, 9}, {1, -1, 4, 1},
     {1, -6, 4, 3}},
};
const int kHStep[2] = {4, 10};
const int kHJ[2] = {4, 7};
const int kLimbClasses[] = {1, 2, 3, 4, 5, 6, 8, 12, 17};

constexpr uint64_t kModulusLimit = 1ull << 54;

int limb_class(uint32_t P) {
  const int Lq = (int)((P + 63u) / 64u);
  for (int c : kLimbClasses)
    if (c >= Lq) return c;
  return -1;
}

// first index of series j whose exponent d + c - step k is negative
uint64_t first_tail(const HostSeries &s, int step, uint64_t d) {
  const int64_t dc = (int64_t)d + s.c;
  return dc < 0 ? 0 : (uint64_t)(dc / step) + 1u;
}

// first index past which every truncated tail term is 0: t >= 1 needs
// P + E >= 0, i.e. k <= (d + c + P) / step
uint64_t first_zero(const HostSeries &s, int step, uint64_t d, uint32_t P) {
  const int64_t v = (int64_t)d + s.c + (int64_t)P;
  return v < 0 ? 0 : (uint64_t)(v / step) + 1u;
}

// Fill a plan for series set `jmask` of `formula` over index range [k0, k1).
int make_plan(int formula, uint64_t n, uint32_t w, uint32_t P, uint32_t jmask, uint64_t k0,
              uint64_t k1, QueryPlan *qp) {
  if (formula != PI_BBP && formula != PI_BELLARD) return PI_EINVAL;
  if (n == 0 || w == 0 || P == 0 || P < w || P > PI_MAX_P || k0 > k1) return PI_EINVAL;
  if (n >= (1ull << 62) - PI_MAX_P - 64) return PI_EUNSUPPORTED;
  memset(qp, 0, sizeof(*qp));
  qp->formula = formula;
  qp->d = n - 1;
  qp->P = P;
  qp->w = w;
  qp->Lq = (P + 63u) / 64u;
  qp->Lk = limb_class(P);
  const int step = kHStep[formula];
  for (int j = 0; j < kHJ[formula]; ++j) {
    if (!(jmask & (1u << j))) continue;
    const HostSeries &s = kHSeries[formula][j];
    const uint64_t kt = first_tail(s, step, qp->d);
    const uint64_t kz = std::max(kt, first_zero(s, step, qp->d, P));
    qp->hk0[j] = std::min(k0, kt);
    qp->hk1[j] = std::min(k1, kt);
    qp->tk0[j] = std::min(std::max(k0, kt), kz);
    qp->tk1[j] = std::max(qp->tk0[j], std::min(k1, kz));
    // largest index whose modulus is used: ends of the non-empty ranges only
    const uint64_t hi = std::max(qp->hk1[j] > qp->hk0[j] ? qp->hk1[j] : 0,
                                 qp->tk1[j] > qp->tk0[j] ? qp->tk1[j] : 0);
    if (hi > 0 && (hi - 1) > (kModulusLimit - s.b) / s.a) return PI_EUNSUPPORTED;
    qp->nhead += qp->hk1[j] - qp->hk0[j];
  }
  return PI_OK;
}

// Arithmetic of the head terms (pi_set_arith): PI_ARITH_FAST uses exact
// binary64 residues where they are cheapest, PI_ARITH_INTEGER integer
// Montgomery arithmetic everywhere. Both give the same bits. The mode is the
// calling host thread's own, so one thread's choice never changes how
// another thread's queries are planned.
thread_local int g_arith = PI_ARITH_FAST;

// Head segments of a plan, split by modulus range.
//  * PI_ARITH_FAST: below 2^22 (R = 2^32, Montgomery one by doublings,
//    three-bit windows), [2^22, 2^27) and [2^27, 2^29) (R = 2^32, run-quotient
//    start, two- and one-bit windows), [2^29, 2^33), [2^33, 2^42) and
//    [2^42, 2^48) (binary64 with four-, three- and two-bit windows),
//    [2^48, 2^51) (binary64, five-bit windows, each digit applied after the
//    window's squarings)
//    and from 2^51 (R = 2^62).
//  * PI_ARITH_INTEGER: the same below 2^29, [2^29, 2^31) (R = 2^32, reduced
//    residues), then R = 2^62 split at 2^36 so that the small moduli, where a
//    lane run's start value has the most slack to cover, do not limit the
//    run length and start bits of the rest.
int head_segments(const QueryPlan &qp, uint32_t acc_off, HeadSeg *out) {
  static const uint64_t kFastLim[7] = {1ull << 22, 1ull << 27, 1ull << 29, 1ull << 33,
                                       1ull << 42, 1ull << 48, 1ull << 51};
  static const uint32_t kFastCls[8] = {22, 27, 29, 33, 42, 48, 51, 64};
  static const uint64_t kIntLim[5] = {1ull << 22, 1ull << 27, 1ull << 29, 1ull << 31, 1ull << 36};
  static const uint32_t kIntCls[6] = {22, 27, 29, 31, 64, 64};
  const bool fast = g_arith == PI_ARITH_FAST;
  const uint64_t *lim = fast ? kFastLim : kIntLim;
  const uint32_t *cls = fast ? kFastCls : kIntCls;
  const int ncls = fast ? 8 : 6;
  int nseg = 0;
  for (int j = 0; j < kHJ[qp.formula]; ++j) {
    const HostSeries &s = kHSeries[qp.formula][j];
    const uint64_t kb = qp.hk0[j], ke = qp.hk1[j];
    if (kb >= ke) continue;
    auto first_k = [&](uint64_t Mlim) {  // first k with a k + b >= Mlim
      const uint64_t k = Mlim > s.b ? (Mlim - s.b + s.a - 1) / s.a : 0;
      return std::min(std::max(k, kb), ke);
    };
    uint64_t cuts[9];
    cuts[0] = kb;
    for (int c = 1; c < ncls; ++c) cuts[c] = first_k(lim[c - 1]);
    cuts[ncls] = ke;
    HeadSeg g;
    memset(&g, 0, sizeof g);
    g.d = qp.d;
    g.formula = (uint32_t)qp.formula;
    g.j = (uint32_t)j;
    g.P = qp.P;
    g.acc_off = acc_off;
    for (int c = 0; c < ncls; ++c) {
      if (cuts[c] >= cuts[c + 1]) continue;
      g.kb = cuts[c];
      g.ke = cuts[c + 1];
      g.cls = cls[c];
      out[nseg++] = g;
    }
  }
  return nseg;
}

void head_segments(const QueryPlan &qp, uint32_t acc_off, std::vector<HeadSeg> &out) {
  HeadSeg segs[kMaxArgSegs];
  const int n = head_segments(qp, acc_off, segs);
  out.insert(out.end(), segs, segs + n);
}

FinQuery fin_query(const QueryPlan &qp, uint64_t out_off, uint32_t status_mode, uint32_t sidx,
                   uint32_t acc_off) {
  FinQuery f;
  memset(&f, 0, sizeof f);
  f.d = qp.d;
  f.nhead = qp.nhead;
  f.out_off = out_off;
  for (int j = 0; j < 7; ++j) {
    f.tk0[j] = qp.tk0[j];
    f.tk1[j] = qp.tk1[j];
  }
  f.formula = (uint32_t)qp.formula;
  f.P = qp.P;
  f.w = qp.w;
  f.Lq = qp.Lq;
  f.want_status = status_mode;
  f.status_idx = sidx;
  f.acc_off = acc_off;
  return f;
}

// ---- device facts and scratch ----------------------------------------------

std::mutex g_mu;
std::map<int, int> g_cus;
struct Arena {
  void *dev = nullptr;
  size_t bytes = 0;
};
std::map<std::pair<int, hipStream_t>, Arena> g_arena;

// Pinned host staging for the tables a batch uploads, one per (device,
// stream). Before it is rewritten, the previous upload from it must be done:
// an event recorded after that upload is waited on.
struct Stage {
  void *host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
std::map<std::pair<int, hipStream_t>, Stage> g_stage;

void *stage(hipStream_t st, size_t bytes, Stage **out, int *err) {
  int dev = 0;
  *err = PI_OK;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = PI_EDEVICE;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Stage &s = g_stage[{dev, st}];
  if (!s.done && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
    *err = PI_EDEVICE;
    return nullptr;
  }
  if (s.pending && hipEventSynchronize(s.done) != hipSuccess) {
    *err = PI_EDEVICE;
    return nullptr;
  }
  s.pending = false;
  if (s.bytes < bytes) {
    if (s.host) (void)hipHostFree(s.host);
    s.host = nullptr;
    s.bytes = 0;
    const size_t nb = std::max(bytes, (size_t)1 << 16);
    if (hipHostMalloc(&s.host, nb, hipHostMallocDefault) != hipSuccess) {
      *err = PI_ENOMEM;
      return nullptr;
    }
    s.bytes = nb;
  }
  *out = &s;
  return s.host;
}

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cus.find(dev);
  if (it != g_cus.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  g_cus[dev] = cus;
  return cus;
}

// Per-(device, stream) scratch, grown on demand. Growing waits for the
// stream so that no queued kernel still uses the old block.
void *arena(hipStream_t st, size_t bytes, int *err) {
  int dev = 0;
  *err = PI_OK;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = PI_EDEVICE;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Arena &a = g_arena[{dev, st}];
  if (a.bytes < bytes) {
    if (a.dev) {
      if (hipStreamSynchronize(st) != hipSuccess || hipFree(a.dev) != hipSuccess) {
        *err = PI_EDEVICE;
        return nullptr;
      }
      a.dev = nullptr;
      a.bytes = 0;
    }
    const size_t nb = std::max(bytes, (size_t)1 << 16);
    if (hipMalloc(&a.dev, nb) != hipSuccess) {
      *err = PI_ENOMEM;
      return nullptr;
    }
    a.bytes = nb;
  }
  return a.dev;
}

// Launch shape per kernel limb class: workgroups per CU (0: as many as fit,
// from the occupancy API) and the cap on indices per lane per chunk. Set by
// pi_set_tuning (e.g. from the autotuner's cache). Entry 0 is the fused launch
// of queries of 1 to kFusedMaxL limbs (batches, serving steps).
struct Tuning {
  uint32_t wg_per_cu = 0;
  uint32_t run_cap = 2048;
};
Tuning g_tune[PI_MAX_L + 1];
std::map<std::pair<int, int>, int> g_occ;  // (device, 2 Lk + by_value) -> workgroups per CU

// Chunk length per lane: long runs amortize the per-chunk fold, but a small
// query still has to fill every workgroup slot several times over. A query's
// carry-save counters take one value below 2^32 per chunk, so its chunk count
// must stay below 2^31: very large queries get longer runs.
uint32_t pick_run(uint64_t head_terms, int grid, uint32_t cap) {
  const uint64_t per = head_terms / (256ull * (uint64_t)grid * 4ull);
  const uint64_t floor_run = head_terms / (256ull << 31) + 1u;
  return (uint32_t)std::max<uint64_t>(floor_run, std::min<uint64_t>(cap, std::max<uint64_t>(1, per)));
}

uint32_t run_cap_for(int Lk) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tune[Lk].run_cap;
}

uint32_t run_cap_fused() { return run_cap_for(0); }

// Grid of the fused launch (queries of 1 to kFusedMaxL limbs): CUs x the
// workgroups per CU its occupancy allows.
int resident_grid_fused() {
  const int cus = device_cus();
  if (cus <= 0) return 2048;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int occ = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_occ.find({dev, 0});
    if (it != g_occ.end()) occ = it->second;
  }
  if (occ == 0) {
    occ = std::max(1, head_occupancy_fused());
    std::lock_guard<std::mutex> lk(g_mu);
    g_occ[{dev, 0}] = occ;
  }
  uint32_t per = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    per = g_tune[0].wg_per_cu;
  }
  return cus * (per ? (int)per : occ);
}

// Grid of a head launch for limb class Lk: CUs x workgroups per CU, from the
// occupancy of the kernel instance that runs it (by_value: segment table in
// the kernel arguments, one query; otherwise in device memory, batches and
// serving steps).
int resident_grid(int Lk, bool by_value) {
  const int cus = device_cus();
  if (cus <= 0) return 2048;
  int dev = 0;
  (void)hipGetDevice(&dev);
  uint32_t per = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    per = g_tune[Lk].wg_per_cu;
  }
  if (per == 0) {
    int occ = 0;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      auto it = g_occ.find({dev, 2 * Lk + (by_value ? 1 : 0)});
      if (it != g_occ.end()) occ = it->second;
    }
    if (occ == 0) {
      occ = std::max(1, head_occupancy(Lk, by_value));
      std::lock_guard<std::mutex> lk(g_mu);
      g_occ[{dev, 2 * Lk + (by_value ? 1 : 0)}] = occ;
    }
    per = (uint32_t)occ;
  }
  return cus * (int)per;
}

int hip_err(hipError_t e) { return e == hipSuccess ? PI_OK : PI_EDEVICE; }

// Largest run (indices per lane per chunk) a class-62 segment with moduli in
// [Mmin, Mmax] and modulus step a allows. A lane's ladder starts from
// g = 2^62 - qM with q = floor(2^62/M_last), so g < (e+1)M with
// e + 1 <= 2^63 a run / M^2 + 2. The first squaring needs g^2 < 2^62 M (its
// output then stays below 8M) and g < 2^57 (digit bounds); with a margin of
// 4 and 2 this asks (e+1)^2 M < 2^60 and (e+1) M < 2^56. Both bounds are
// largest at an end of the modulus range.
uint32_t safe_run62(uint32_t run, uint64_t Mmin, uint64_t Mmax, uint64_t a, uint32_t pre = 0) {
  const double shift = std::ldexp(1.0, (int)((1u << pre) - 1u));  // largest 2^v
  auto ok = [&](double r) {
    const double A = std::ldexp((double)a * r, 63);
    for (double M : {(double)Mmin, (double)Mmax}) {
      const double g = (A / (M * M) + 2.0) * M * shift;
      if (g * g >= std::ldexp(M, 60) || g >= std::ldexp(1.0, 56)) return false;
    }
    return true;
  };
  while (run > 1 && !ok((double)run)) run = std::max<uint32_t>(1, run / 2);
  return ok((double)run) ? run : 0;
}

// Exponent bits a class-62 segment can fold into its start value at `run`
// (0..3): the largest count whose biggest shift keeps the bounds.
uint32_t safe_pre62(uint32_t run, uint64_t Mmin, uint64_t Mmax, uint64_t a) {
  for (uint32_t pre = 3; pre > 0; --pre)
    if (safe_run62(run, Mmin, Mmax, a, pre) == run) return pre;
  return 0;
}

// Number the chunks of one query's segments and fix each segment's run: about
// a quarter of the segment per lane-run column up to run_cap, and for the
// run-quotient and class-62 starts no more than their start-value bounds
// allow. Runs held down by those bounds add chunks, so the cap doubles until
// the query has fewer than 2^31 chunks: its carry-save counters take one
// value below 2^32 per chunk and stay exact below 2^32 of them.
uint64_t number_chunks(HeadSeg *segs, size_t nseg, uint32_t run_cap, uint64_t chunk_base) {
  for (;;) {
    uint64_t nchunks = chunk_base;
    for (size_t i = 0; i < nseg; ++i) {
      HeadSeg &g = segs[i];
      const HostSeries &s = kHSeries[g.formula][g.j];
      const uint64_t len = g.ke - g.kb;
      uint32_t run = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(run_cap, len / 1024u));
      g.pre = 0;
      if (g.cls == 27 || g.cls == 29 || g.cls == 31) {
        // the start value 2^32 - qM stays below 2M when 2^32 2a run < Mmin^2
        const uint64_t Mmin = s.a * g.kb + s.b;
        const uint64_t lim = (uint64_t)(((unsigned __int128)Mmin * Mmin >> 32) / (2u * s.a));
        run = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(run, lim));
      }
      if (g.cls == 64) {
        const uint64_t Mmin = s.a * g.kb + s.b, Mmax = s.a * (g.ke - 1) + s.b;
        run = std::max<uint32_t>(1, safe_run62(run, Mmin, Mmax, s.a));
        g.pre = safe_pre62(run, Mmin, Mmax, s.a);
      }
      g.run = run;
      g.chunk0 = nchunks;
      nchunks += (len + 256ull * run - 1) / (256ull * run);
    }
    if (nchunks - chunk_base < (1ull << 31) || run_cap >= (1u << 30)) return nchunks - chunk_base;
    run_cap *= 2;
  }
}

uint64_t number_chunks(std::vector<HeadSeg> &segs, uint32_t run_cap, uint64_t chunk_base) {
  return number_chunks(segs.data(), segs.size(), run_cap, chunk_base);
}

// Smallest run cap that keeps a query below 2^31 chunks (its counters take one
// value below 2^32 per chunk).
uint32_t min_run_cap(uint64_t head_terms) {
  return (uint32_t)(head_terms / (256ull << 31) + 1u);
}

// Launch everything for one planned query (head segments passed by value).
// Its scratch is 2Lk carry-save counters and then the head launch's chunk
// counter: the library's per-stream arena, or `scratch` when given (at least
// 2Lk + 1 words, nothing is allocated then).
int run_single(const QueryPlan &qp, uint64_t *out, pi_status *status, uint32_t mode,
               hipStream_t st, unsigned long long *scratch = nullptr) {
  HeadSegTable tab;
  memset(&tab, 0, sizeof tab);
  tab.n = head_segments(qp, 0, tab.s);
  const int grid_max = resident_grid(qp.Lk, true);
  const uint64_t nchunks =
      number_chunks(tab.s, (size_t)tab.n, pick_run(qp.nhead, grid_max, run_cap_for(qp.Lk)), 0);
  const int Lk = qp.Lk;
  int err = PI_OK;
  auto *acc = scratch ? scratch
                      : (unsigned long long *)arena(
                            st, (2u * PI_MAX_L + 1u) * sizeof(unsigned long long), &err);
  if (!acc) return err;
  if (int e = hip_err(launch_zero(acc, 2u * (uint64_t)Lk + 1u, st))) return e;
  if (nchunks) {
    const int grid = (int)std::min<uint64_t>(nchunks, (uint64_t)grid_max);
    if (int e = hip_err(launch_head_args(Lk, tab, nchunks, grid, acc, acc + 2u * Lk, st)))
      return e;
  }
  FinQuery fq = fin_query(qp, 0, status != nullptr ? mode : 0u, 0, 0);
  return hip_err(launch_finalize(Lk, fq, nullptr, 1, acc, out, status, st));
}

// ---- batches -------------------------------------------------------------

// One launch group of a batch: every query of 1 to kFusedMaxL limbs in the
// fused kernel (Lk = 0), or the queries of one larger limb class; their head
// segments and finalize records, and where each lives in the workspace.
struct ClassPlan {
  int Lk = 0;
  int grid = 2048;  // head launch grid, fixed at planning
  std::vector<HeadSeg> segs;
  std::vector<FinQuery> fins;
  uint64_t nchunks = 0;
  uint32_t acc_words = 0;  // the queries' carry-save counters, 2 Lk each
  size_t acc_off = 0, seg_off = 0, fin_off = 0;
};
struct BatchPlan {
  std::vector<ClassPlan> cls;
  size_t bytes = 0;
};

size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

int plan_batch(const pi_query *q, int count, BatchPlan *bp) {
  if (count < 0 || (count > 0 && !q)) return PI_EINVAL;
  std::map<int, int> by_class;  // launch group (0: fused) -> index in bp->cls
  for (int i = 0; i < count; ++i) {
    if (q[i].reserved != 0) return PI_EINVAL;
    QueryPlan qp;
    if (int e = make_plan(q[i].formula, q[i].n, q[i].nbits, q[i].P, 0x7fu, 0, UINT64_MAX, &qp))
      return e;
    const int group = qp.Lk <= kFusedMaxL ? 0 : qp.Lk;
    auto it = by_class.find(group);
    if (it == by_class.end()) {
      it = by_class.emplace(group, (int)bp->cls.size()).first;
      bp->cls.emplace_back();
      bp->cls.back().Lk = group;
      bp->cls.back().grid = group ? resident_grid(group, false) : resident_grid_fused();
    }
    ClassPlan &c = bp->cls[it->second];
    const uint32_t local = c.acc_words;
    c.acc_words += 2u * (uint32_t)qp.Lk;
    std::vector<HeadSeg> segs;
    head_segments(qp, local, segs);
    const uint32_t cap = std::max(
        pick_run(qp.nhead, c.grid, group ? run_cap_for(qp.Lk) : run_cap_fused()),
        min_run_cap(qp.nhead));
    c.nchunks += number_chunks(segs, cap, c.nchunks);
    c.segs.insert(c.segs.end(), segs.begin(), segs.end());
    c.fins.push_back(fin_query(qp, q[i].out_offset, 1u, (uint32_t)i, local));
  }
  size_t off = 0;
  for (ClassPlan &c : bp->cls) {
    c.acc_off = off;  // carry-save counters of each query, then the chunk counter
    off = align256(off + ((size_t)c.acc_words + 1u) * sizeof(unsigned long long));
    c.seg_off = off;
    off = align256(off + c.segs.size() * sizeof(HeadSeg));
    c.fin_off = off;
    off = align256(off + c.fins.size() * sizeof(FinQuery));
  }
  bp->bytes = std::max<size_t>(off, 256);
  return PI_OK;
}

int launch_planned(const BatchPlan &bp, char *ws, uint64_t *out, pi_status *status,
                   hipStream_t st);

// Upload the tables (through pinned staging), clear the counters, then one
// head launch and one finalize launch per limb class, all on `st`.
int run_batch(BatchPlan &bp, char *ws, uint64_t *out, pi_status *status, hipStream_t st) {
  size_t table_bytes = 0;
  for (ClassPlan &c : bp.cls) {
    for (FinQuery &f : c.fins) f.want_status = status != nullptr ? 1u : 0u;
    table_bytes += c.segs.size() * sizeof(HeadSeg) + c.fins.size() * sizeof(FinQuery);
  }
  Stage *sg = nullptr;
  int err = PI_OK;
  char *host = (char *)stage(st, table_bytes, &sg, &err);
  if (!host) return err;
  size_t hoff = 0;
  for (const ClassPlan &c : bp.cls) {
    auto *segs = (HeadSeg *)(ws + c.seg_off);
    auto *fins = (FinQuery *)(ws + c.fin_off);
    const size_t sb = c.segs.size() * sizeof(HeadSeg), fb = c.fins.size() * sizeof(FinQuery);
    memcpy(host + hoff, c.segs.data(), sb);
    memcpy(host + hoff + sb, c.fins.data(), fb);
    if (sb && hipMemcpyAsync(segs, host + hoff, sb, hipMemcpyHostToDevice, st) != hipSuccess)
      return PI_EDEVICE;
    if (hipMemcpyAsync(fins, host + hoff + sb, fb, hipMemcpyHostToDevice, st) != hipSuccess)
      return PI_EDEVICE;
    hoff += sb + fb;
  }
  if (hipEventRecord(sg->done, st) != hipSuccess) return PI_EDEVICE;
  sg->pending = true;
  return launch_planned(bp, ws, out, status, st);
}

}  // namespace host
}  // namespace pibbp

using namespace pibbp;
using namespace pibbp::host;

extern "C" {

int pi_extract_ex(int formula, uint64_t n, uint32_t nbits, uint32_t P, uint64_t *out,
                  pi_status *status, hipStream_t stream) {
  if (!out) return PI_EINVAL;
  QueryPlan qp;
  if (int e = make_plan(formula, n, nbits, P, 0x7fu, 0, UINT64_MAX, &qp)) return e;
  return run_single(qp, out, status, 1u, stream);
}

int pi_extract_noalloc(int formula, uint64_t n, uint32_t nbits, uint32_t P, uint64_t *out,
                       pi_status *status, hipStream_t stream) {
  if (!out) return PI_EINVAL;
  QueryPlan qp;
  if (int e = make_plan(formula, n, nbits, P, 0x7fu, 0, UINT64_MAX, &qp)) return e;
  unsigned long long *scratch = nullptr;
  uint32_t words = 0;
  if (static_scratch(&scratch, &words) != hipSuccess) return PI_EDEVICE;
  if (2u * (uint32_t)qp.Lk + 1u > words) return PI_ESCRATCH;
  return run_single(qp, out, status, 1u, stream, scratch);
}

int pi_extract(int formula, uint64_t n, uint32_t nbits, uint64_t *out, hipStream_t stream) {
  if (nbits == 0 || nbits > PI_MAX_P - 64) return PI_EINVAL;
  return pi_extract_ex(formula, n, nbits, nbits + 64u, out, nullptr, stream);
}

int pi_sum_slice(int term, uint64_t n, uint64_t k0, uint64_t k1, uint32_t P, uint64_t *out,
                 hipStream_t stream) {
  if (!out || term < 0) return PI_EINVAL;
  const int formula = term / 16, j = term % 16;
  if ((formula != PI_BBP && formula != PI_BELLARD) || j >= kHJ[formula]) return PI_EINVAL;
  QueryPlan qp;
  if (int e = make_plan(formula, n, P, P, 1u << j, k0, k1, &qp)) return e;
  return run_single(qp, out, nullptr, 0u, stream);
}

int pi_sum_slice_ex(int term, uint64_t n, uint64_t k0, uint64_t k1, uint32_t P, uint64_t *out,
                    pi_status *status, hipStream_t stream) {
  if (!out || term < 0) return PI_EINVAL;
  const int formula = term / 16, j = term % 16;
  if ((formula != PI_BBP && formula != PI_BELLARD) || j >= kHJ[formula]) return PI_EINVAL;
  QueryPlan qp;
  if (int e = make_plan(formula, n, P, P, 1u << j, k0, k1, &qp)) return e;
  return run_single(qp, out, status, 2u, stream);
}

int pi_combine(const uint64_t *parts, int count, uint32_t P, uint32_t nbits, uint32_t nseries,
               uint64_t nterms, uint64_t *out, pi_status *status, hipStream_t stream) {
  if (!out || count < 0 || (count > 0 && !parts) || P == 0 || P > PI_MAX_P || nbits == 0 ||
      nbits > P)
    return PI_EINVAL;
  return hip_err(launch_combine(parts, count, (int)((P + 63u) / 64u), P, nbits, nterms, nseries,
                                out, status, stream));
}

uint64_t pi_head_terms(int formula, uint64_t n) {
  if ((formula != PI_BBP && formula != PI_BELLARD) || n == 0) return 0;
  uint64_t tot = 0;
  for (int j = 0; j < kHJ[formula]; ++j)
    tot += first_tail(kHSeries[formula][j], kHStep[formula], n - 1);
  return tot;
}

int pi_plan_head(int formula, uint32_t series_mask, uint64_t n, uint64_t k0, uint64_t k1,
                 uint32_t P, pi_segment *segs, int max_segs, int *count) {
  if (!count || max_segs < 0 || (max_segs > 0 && !segs)) return PI_EINVAL;
  if (formula != PI_BBP && formula != PI_BELLARD) return PI_EINVAL;
  QueryPlan qp;
  if (int e = make_plan(formula, n, P, P, series_mask, k0, k1, &qp)) return e;
  std::vector<HeadSeg> hs;
  head_segments(qp, 0, hs);
  number_chunks(hs, pick_run(qp.nhead, resident_grid(qp.Lk, true), run_cap_for(qp.Lk)), 0);
  *count = (int)hs.size();
  if ((int)hs.size() > max_segs) return PI_EINVAL;
  for (size_t i = 0; i < hs.size(); ++i) {
    const HeadSeg &g = hs[i];
    const uint64_t next = i + 1 < hs.size() ? hs[i + 1].chunk0 : 0;
    pi_segment &o = segs[i];
    o.j = g.j;
    o.cls = g.cls;
    o.run = g.run;
    o.pre = g.pre;
    o.kb = g.kb;
    o.ke = g.ke;
    o.nchunks = i + 1 < hs.size() ? next - g.chunk0
                                  : (g.ke - g.kb + 256ull * g.run - 1) / (256ull * g.run);
  }
  return PI_OK;
}

}  // extern "C"

struct pi_batch {
  BatchPlan bp;
  char *ws = nullptr;
  uint64_t *out = nullptr;
  pi_status *status = nullptr;
  hipEvent_t last = nullptr;  // recorded after each launch that is not being captured
  bool recorded = false;
};

namespace pibbp {
namespace host {
// Kernel launches of a planned batch whose tables are already on the device.
int launch_planned(const BatchPlan &bp, char *ws, uint64_t *out, pi_status *status,
                   hipStream_t st) {
  for (const ClassPlan &c : bp.cls) {
    const int grid_max = c.grid;
    auto *acc = (unsigned long long *)(ws + c.acc_off);
    auto *segs = (HeadSeg *)(ws + c.seg_off);
    auto *fins = (FinQuery *)(ws + c.fin_off);
    const uint64_t ncount = c.acc_words;
    if (int e = hip_err(launch_zero(acc, ncount + 1u, st))) return e;
    if (c.nchunks) {
      const int grid = (int)std::min<uint64_t>(c.nchunks, (uint64_t)grid_max);
      const hipError_t he =
          c.Lk ? launch_head_ptr(c.Lk, segs, (int)c.segs.size(), c.nchunks, grid, acc,
                                 acc + ncount, st)
               : launch_head_fused(segs, (int)c.segs.size(), c.nchunks, grid, acc, acc + ncount,
                                   st);
      if (int e = hip_err(he)) return e;
    }
    FinQuery none;
    memset(&none, 0, sizeof none);
    const hipError_t fe =
        c.Lk ? launch_finalize(c.Lk, none, fins, (int)c.fins.size(), acc, out, status, st)
             : launch_finalize_fused(fins, (int)c.fins.size(), acc, out, status, st);
    if (int e = hip_err(fe)) return e;
  }
  return PI_OK;
}
}  // namespace host
}  // namespace pibbp

extern "C" {

int pi_batch_create(const pi_query *q, int count, uint64_t *out, pi_status *status,
                    pi_batch **plan) {
  if (!plan || count <= 0 || !q || !out) return PI_EINVAL;
  *plan = nullptr;
  pi_batch *b = new pi_batch();
  if (int e = plan_batch(q, count, &b->bp)) {
    delete b;
    return e;
  }
  for (ClassPlan &c : b->bp.cls)
    for (FinQuery &f : c.fins) f.want_status = status != nullptr ? 1u : 0u;
  if (hipMalloc((void **)&b->ws, b->bp.bytes) != hipSuccess) {
    delete b;
    return PI_ENOMEM;
  }
  for (const ClassPlan &c : b->bp.cls) {
    if ((!c.segs.empty() && hipMemcpy(b->ws + c.seg_off, c.segs.data(),
                                      c.segs.size() * sizeof(HeadSeg),
                                      hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(b->ws + c.fin_off, c.fins.data(), c.fins.size() * sizeof(FinQuery),
                  hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(b->ws);
      delete b;
      return PI_EDEVICE;
    }
  }
  if (hipEventCreateWithFlags(&b->last, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(b->ws);
    delete b;
    return PI_EDEVICE;
  }
  b->out = out;
  b->status = status;
  *plan = b;
  return PI_OK;
}

int pi_batch_launch(pi_batch *plan, hipStream_t stream) {
  if (!plan) return PI_EINVAL;
  if (int e = launch_planned(plan->bp, plan->ws, plan->out, plan->status, stream)) return e;
  // an eager launch is marked for pi_batch_destroy; under capture the graph's
  // replays are the caller's to finish first
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return PI_EDEVICE;
  if (cs == hipStreamCaptureStatusNone) {
    if (hipEventRecord(plan->last, stream) != hipSuccess) return PI_EDEVICE;
    plan->recorded = true;
  }
  return PI_OK;
}

void pi_batch_destroy(pi_batch *plan) {
  if (!plan) return;
  if (plan->recorded) (void)hipEventSynchronize(plan->last);
  if (plan->last) (void)hipEventDestroy(plan->last);
  (void)hipFree(plan->ws);
  delete plan;
}

size_t pi_workspace_size(const pi_query *q, int count) {
  BatchPlan bp;
  if (plan_batch(q, count, &bp) != PI_OK) return 0;
  return bp.bytes;
}

int pi_extract_batch(const pi_query *q, int count, uint64_t *out, pi_status *status,
                     void *workspace, size_t ws_bytes, hipStream_t stream) {
  if (count < 0 || (count > 0 && (!q || !out))) return PI_EINVAL;
  if (count == 0) return PI_OK;
  BatchPlan bp;
  if (int e = plan_batch(q, count, &bp)) return e;
  char *ws = (char *)workspace;
  if (ws) {
    if (ws_bytes < bp.bytes) return PI_EINVAL;
  } else {
    int err = PI_OK;
    ws = (char *)arena(stream, bp.bytes, &err);
    if (!ws) return err;
  }
  return run_batch(bp, ws, out, status, stream);
}

int pi_set_arith(int mode) {
  if (mode != PI_ARITH_FAST && mode != PI_ARITH_INTEGER) return PI_EINVAL;
  g_arith = mode;
  return PI_OK;
}

int pi_get_arith(void) { return g_arith; }

int pi_set_tuning(int limbs, uint32_t wg_per_cu, uint32_t run_cap) {
  if (limbs < PI_TUNE_FUSED || limbs > PI_MAX_L || run_cap == 0 || run_cap > 4096 ||
      wg_per_cu > 64)
    return PI_EINVAL;
  const int cls = limbs <= 0 ? 0 : limb_class(64u * (uint32_t)limbs);
  std::lock_guard<std::mutex> lk(g_mu);
  for (int L = 0; L <= PI_MAX_L; ++L)
    if ((limbs == 0) || (limbs == PI_TUNE_FUSED && L == 0) || (limbs > 0 && L == cls)) {
      g_tune[L].wg_per_cu = wg_per_cu;
      g_tune[L].run_cap = run_cap;
    }
  return PI_OK;
}

int pi_get_tuning(int limbs, uint32_t *wg_per_cu, uint32_t *run_cap) {
  if (limbs < PI_TUNE_FUSED || limbs == 0 || limbs > PI_MAX_L || !wg_per_cu || !run_cap)
    return PI_EINVAL;
  const int cls = limbs == PI_TUNE_FUSED ? 0 : limb_class(64u * (uint32_t)limbs);
  std::lock_guard<std::mutex> lk(g_mu);
  *wg_per_cu = g_tune[cls].wg_per_cu;
  *run_cap = g_tune[cls].run_cap;
  return PI_OK;
}

const char *pi_strerror(int code) {
  switch (code) {
    case PI_OK: return "ok";
    case PI_UNCERTAIN: return "bits computed exactly but not certified by the guard window";
    case PI_EINVAL: return "invalid argument";
    case PI_ENOMEM: return "out of device memory";
    case PI_EDEVICE: return "HIP runtime or device error";
    case PI_EUNSUPPORTED: return "outside the supported range (modulus >= 2^54 or n too large)";
    case PI_ESCRATCH: return "needs more than the static scratch of pi_extract_noalloc";
    default: return "unknown error code";
  }
}

void pi_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &kv : g_arena) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(kv.first.first);
    (void)hipStreamSynchronize(kv.first.second);
    (void)hipFree(kv.second.dev);
    (void)hipSetDevice(cur);
  }
  g_arena.clear();
  for (auto &kv : g_stage) {
    if (kv.second.pending) (void)hipEventSynchronize(kv.second.done);
    if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    if (kv.second.host) (void)hipHostFree(kv.second.host);
  }
  g_stage.clear();
}

}  // extern "C"
