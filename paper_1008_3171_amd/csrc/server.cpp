// Continuous-batching server (the pi_server_* C ABI).
//
// Section 4.3 of the paper keeps a cluster busy by submitting small jobs
// whenever map or reduce slots are idle, and section 4 keeps every partial
// sum persisted so work can stop and resume. On one GPU the same two ideas
// become: admit a query whenever a device slot is free, give every active
// query a share of each step's head terms, and keep each query's partial sum
// (its carry-save counters) in its device slot between steps. A query
// finishes when its last chunk has run; it is then finalized (tail,
// normalization, certification) and its result is copied to the host.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "host.h"
#include "pibbp.h"
#include "plan.h"

using namespace pibbp;
using namespace pibbp::host;

namespace {

constexpr uint32_t kSlotCounters = 2u * PI_MAX_L;  // carry-save counters per slot
constexpr uint32_t kChunkCounters = 16;             // one per head launch of a step (<= 9)

struct Active {
  uint64_t tag = 0;
  QueryPlan qp{};
  std::vector<HeadSeg> segs;  // chunk0 counted from the query's first chunk
  uint64_t nchunks = 0;
  uint64_t next = 0;          // first chunk not yet launched
  size_t seg = 0;             // segment holding chunk `next`
  uint32_t slot = 0;
};

uint64_t seg_chunks(const HeadSeg &g) {
  const uint64_t ch = 256ull * g.run;
  return (g.ke - g.kb + ch - 1) / ch;
}

}  // namespace

struct pi_server {
  hipStream_t st = nullptr;
  uint32_t cap = 0;
  uint64_t step_terms = 0;
  unsigned long long *acc = nullptr;  // cap x kSlotCounters, then kChunkCounters
  uint64_t *res = nullptr;            // cap x PI_MAX_L limbs, rows in finish order
  pi_status *res_st = nullptr;        // cap
  HeadSeg *dsegs = nullptr;
  size_t dsegs_cap = 0;
  FinQuery *dfins = nullptr;
  size_t dfins_cap = 0;
  char *pinned = nullptr;             // host staging: tables, then results
  size_t pinned_bytes = 0;
  std::vector<uint32_t> free_slots;
  std::vector<Active> active;
  std::deque<pi_result> done;
};

namespace {

template <typename T>
int grow_device(T **p, size_t *have, size_t need) {
  if (*have >= need) return PI_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  const size_t n = std::max<size_t>(need, 256);
  if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) return PI_ENOMEM;
  *have = n;
  return PI_OK;
}

int grow_pinned(pi_server *s, size_t need) {
  if (s->pinned_bytes >= need) return PI_OK;
  if (s->pinned) (void)hipHostFree(s->pinned);
  s->pinned = nullptr;
  s->pinned_bytes = 0;
  const size_t n = std::max<size_t>(need, 1 << 16);
  if (hipHostMalloc((void **)&s->pinned, n, hipHostMallocDefault) != hipSuccess) return PI_ENOMEM;
  s->pinned_bytes = n;
  return PI_OK;
}

void release(pi_server *s) {
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->acc) (void)hipFree(s->acc);
  if (s->res) (void)hipFree(s->res);
  if (s->res_st) (void)hipFree(s->res_st);
  if (s->dsegs) (void)hipFree(s->dsegs);
  if (s->dfins) (void)hipFree(s->dfins);
  if (s->pinned) (void)hipHostFree(s->pinned);
}

}  // namespace

extern "C" {

int pi_server_create(uint32_t max_active, uint64_t step_terms, hipStream_t stream,
                     pi_server **out) {
  if (!out || max_active == 0 || step_terms == 0) return PI_EINVAL;
  *out = nullptr;
  // make the caller's device current first: hipMemGetInfo needs its context,
  // and this may be the process's first GPU call
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipSetDevice(dev) != hipSuccess) return PI_EDEVICE;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return PI_EDEVICE;
  // device bytes one slot can need: counters, result row and status, and its
  // share of the step tables (up to kMaxArgSegs segments and one finalize record)
  const size_t per_slot = kSlotCounters * 8u + PI_MAX_L * 8u + sizeof(pi_status) +
                          kMaxArgSegs * sizeof(HeadSeg) + sizeof(FinQuery);
  const uint64_t by_mem = (uint64_t)(free_b / 4u / per_slot);
  const uint32_t cap = (uint32_t)std::min<uint64_t>(max_active, by_mem);
  if (cap == 0) return PI_ENOMEM;
  pi_server *s = new pi_server();
  s->st = stream;
  s->cap = cap;
  s->step_terms = step_terms;
  if (hipMalloc((void **)&s->acc, ((size_t)cap * kSlotCounters + kChunkCounters) * 8u) !=
          hipSuccess ||
      hipMalloc((void **)&s->res, (size_t)cap * PI_MAX_L * 8u) != hipSuccess ||
      hipMalloc((void **)&s->res_st, (size_t)cap * sizeof(pi_status)) != hipSuccess) {
    release(s);
    delete s;
    return PI_ENOMEM;
  }
  s->free_slots.reserve(cap);
  for (uint32_t i = cap; i-- > 0;) s->free_slots.push_back(i);
  *out = s;
  return PI_OK;
}

int pi_server_submit(pi_server *s, const pi_query *q, uint64_t tag) {
  if (!s || !q || q->reserved != 0) return PI_EINVAL;
  Active a;
  if (int e = make_plan(q->formula, q->n, q->nbits, q->P, 0x7fu, 0, UINT64_MAX, &a.qp)) return e;
  if (s->free_slots.empty()) return PI_BUSY;
  a.slot = s->free_slots.back();
  if (int e = hip_err(launch_zero(s->acc + (uint64_t)a.slot * kSlotCounters, kSlotCounters, s->st)))
    return e;
  s->free_slots.pop_back();
  a.tag = tag;
  head_segments(a.qp, a.slot * kSlotCounters, a.segs);
  const uint32_t cap = std::max(pick_run(a.qp.nhead, resident_grid(a.qp.Lk, false), run_cap_for(a.qp.Lk)),
                                min_run_cap(a.qp.nhead));
  a.nchunks = number_chunks(a.segs, cap, 0);
  s->active.push_back(std::move(a));
  return PI_OK;
}

int pi_server_step(pi_server *s, uint32_t *finished) {
  if (!s) return PI_EINVAL;
  if (finished) *finished = 0;
  if (s->active.empty()) return PI_OK;
  // 1. each active query takes chunks worth up to its fair share of terms
  const uint64_t quota = std::max<uint64_t>(1, s->step_terms / s->active.size());
  std::map<int, std::vector<HeadSeg>> segs_by_class;
  std::map<int, uint64_t> chunks_by_class;
  std::vector<size_t> finishing;
  for (size_t i = 0; i < s->active.size(); ++i) {
    Active &a = s->active[i];
    const int Lk = a.qp.Lk;
    uint64_t taken = 0;
    while (a.next < a.nchunks && taken < quota) {
      while (a.seg + 1 < a.segs.size() && a.segs[a.seg + 1].chunk0 <= a.next) ++a.seg;
      const HeadSeg &g = a.segs[a.seg];
      const uint64_t ch = 256ull * g.run;
      const uint64_t end = g.chunk0 + seg_chunks(g);
      const uint64_t want = std::max<uint64_t>(1, (quota - taken + ch - 1) / ch);
      const uint64_t c1 = std::min(end, a.next + want);
      HeadSeg h = g;
      h.kb = g.kb + (a.next - g.chunk0) * ch;
      h.ke = std::min(g.ke, g.kb + (c1 - g.chunk0) * ch);
      h.chunk0 = chunks_by_class[Lk];
      chunks_by_class[Lk] += c1 - a.next;
      segs_by_class[Lk].push_back(h);
      taken += h.ke - h.kb;
      a.next = c1;
    }
    if (a.next == a.nchunks) finishing.push_back(i);
  }
  // 2. finalize records of the queries whose last chunk runs in this step;
  //    their results land in rows 0, 1, ... in finishing order
  std::map<int, std::vector<FinQuery>> fins_by_class;
  for (size_t r = 0; r < finishing.size(); ++r) {
    const Active &a = s->active[finishing[r]];
    fins_by_class[a.qp.Lk].push_back(fin_query(a.qp, (uint64_t)r * PI_MAX_L, 1u, (uint32_t)r,
                                               a.slot * kSlotCounters));
  }
  size_t nsegs = 0, nfins = 0;
  for (auto &kv : segs_by_class) nsegs += kv.second.size();
  for (auto &kv : fins_by_class) nfins += kv.second.size();
  // 3. upload the tables (the stream is idle: the previous step waited)
  const size_t tbytes = nsegs * sizeof(HeadSeg) + nfins * sizeof(FinQuery);
  const size_t rbytes = finishing.size() * (PI_MAX_L * 8u + sizeof(pi_status));
  if (int e = grow_device(&s->dsegs, &s->dsegs_cap, nsegs)) return e;
  if (int e = grow_device(&s->dfins, &s->dfins_cap, nfins)) return e;
  if (int e = grow_pinned(s, tbytes + rbytes)) return e;
  size_t so = 0, fo = 0;
  std::map<int, std::pair<size_t, size_t>> seg_at, fin_at;  // class -> (offset, count)
  for (auto &kv : segs_by_class) {
    memcpy(s->pinned + so * sizeof(HeadSeg), kv.second.data(), kv.second.size() * sizeof(HeadSeg));
    seg_at[kv.first] = {so, kv.second.size()};
    so += kv.second.size();
  }
  char *fhost = s->pinned + nsegs * sizeof(HeadSeg);
  for (auto &kv : fins_by_class) {
    memcpy(fhost + fo * sizeof(FinQuery), kv.second.data(), kv.second.size() * sizeof(FinQuery));
    fin_at[kv.first] = {fo, kv.second.size()};
    fo += kv.second.size();
  }
  if (nsegs && hipMemcpyAsync(s->dsegs, s->pinned, nsegs * sizeof(HeadSeg), hipMemcpyHostToDevice,
                              s->st) != hipSuccess)
    return PI_EDEVICE;
  if (nfins && hipMemcpyAsync(s->dfins, fhost, nfins * sizeof(FinQuery), hipMemcpyHostToDevice,
                              s->st) != hipSuccess)
    return PI_EDEVICE;
  // 4. head launches (each with its own chunk counter, cleared first), then
  //    finalize launches, per limb class
  unsigned long long *ctr = s->acc + (uint64_t)s->cap * kSlotCounters;
  if (!seg_at.empty())
    if (int e = hip_err(launch_zero(ctr, kChunkCounters, s->st))) return e;
  int launch = 0;
  for (auto &kv : seg_at) {
    const int Lk = kv.first;
    const uint64_t nch = chunks_by_class[Lk];
    if (!nch) continue;
    const int grid = (int)std::min<uint64_t>(nch, (uint64_t)resident_grid(Lk, false));
    if (int e = hip_err(launch_head_ptr(Lk, s->dsegs + kv.second.first, (int)kv.second.second, nch,
                                        grid, s->acc, ctr + launch++, s->st)))
      return e;
  }
  FinQuery none;
  memset(&none, 0, sizeof none);
  for (auto &kv : fin_at)
    if (int e = hip_err(launch_finalize(kv.first, none, s->dfins + kv.second.first,
                                        (int)kv.second.second, s->acc, s->res, s->res_st, s->st)))
      return e;
  // 5. bring the finished rows home and wait for the step
  char *rhost = s->pinned + tbytes;
  char *shost = rhost + finishing.size() * PI_MAX_L * 8u;
  if (!finishing.empty()) {
    if (hipMemcpyAsync(rhost, s->res, finishing.size() * PI_MAX_L * 8u, hipMemcpyDeviceToHost,
                       s->st) != hipSuccess ||
        hipMemcpyAsync(shost, s->res_st, finishing.size() * sizeof(pi_status),
                       hipMemcpyDeviceToHost, s->st) != hipSuccess)
      return PI_EDEVICE;
  }
  if (hipStreamSynchronize(s->st) != hipSuccess) return PI_EDEVICE;
  for (size_t r = 0; r < finishing.size(); ++r) {
    const Active &a = s->active[finishing[r]];
    pi_result res;
    memset(&res, 0, sizeof res);
    pi_status stv;
    memcpy(&stv, shost + r * sizeof(pi_status), sizeof stv);
    res.tag = a.tag;
    res.code = stv.code;
    res.P = a.qp.P;
    res.nterms = stv.nterms;
    memcpy(res.limbs, rhost + r * PI_MAX_L * 8u, a.qp.Lq * 8u);
    s->done.push_back(res);
  }
  // 6. retire: free the slots, drop the finished queries
  std::vector<bool> gone(s->active.size(), false);
  for (size_t i : finishing) {
    gone[i] = true;
    s->free_slots.push_back(s->active[i].slot);
  }
  size_t w = 0;
  for (size_t i = 0; i < s->active.size(); ++i)
    if (!gone[i]) {
      if (w != i) s->active[w] = std::move(s->active[i]);
      ++w;
    }
  s->active.resize(w);
  if (finished) *finished = (uint32_t)finishing.size();
  return PI_OK;
}

int pi_server_poll(pi_server *s, pi_result *out, uint32_t max, uint32_t *count) {
  if (!s || !count || (max && !out)) return PI_EINVAL;
  uint32_t n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *count = n;
  return PI_OK;
}

uint32_t pi_server_active(const pi_server *s) { return s ? (uint32_t)s->active.size() : 0; }

uint32_t pi_server_capacity(const pi_server *s) { return s ? s->cap : 0; }

void pi_server_destroy(pi_server *s) {
  if (!s) return;
  release(s);
  delete s;
}

}  // extern "C"
