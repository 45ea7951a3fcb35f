// Continuous-batching server (the pi_server_* C ABI).
//
// Section 4.3 of the paper keeps a cluster busy by submitting small jobs
// whenever map or reduce slots are idle, and section 4 keeps every partial
// sum persisted so work can stop and resume. On one GPU the same two ideas
// become: admit a query whenever a device slot can be had within the
// server's memory budget, give every active query a share of each step's
// head terms, and keep each query's partial sum (its carry-save counters) in
// its device slot between steps. A query finishes when its last chunk has
// run; it is then finalized (tail, normalization, certification) and its
// result is copied to the host.
//
// Steps are pipelined one deep by default: pi_server_step plans and enqueues
// step N and then waits only for step N-1, so the host plans the next step
// while the device runs the current one (pi_server_set_pipeline(s, 0) waits
// for step N as well, which lets a query arriving during a step join the very
// next one, at the cost of the device idling while the host plans). Everything a step touches that the next one
// could overwrite (tables, result rows, host staging, chunk counters) is
// double-buffered by step parity; the carry-save slots are ordered by the
// stream alone.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstddef>
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
constexpr uint32_t kFirstSlots = 64;                // slots allocated at creation (at most)
constexpr uint64_t kStepChunksPerSlot = 8;          // chunks per workgroup slot in a full step

// Device bytes one admitted query can need: its counters, a result row and
// status, and its share of a step's tables (up to kMaxArgSegs segments and
// one finalize record), for each of the two step buffers.
constexpr size_t kSlotBytes = kSlotCounters * 8u +
                              2u * (PI_MAX_L * 8u + sizeof(pi_status) +
                                    kMaxArgSegs * sizeof(HeadSeg) + sizeof(FinQuery));

struct Active {
  uint64_t tag = 0;
  QueryPlan qp{};
  std::vector<HeadSeg> segs;  // chunk0 counted from the query's first chunk
  uint64_t nchunks = 0;
  uint64_t next = 0;          // first chunk not yet launched
  size_t seg = 0;             // segment holding chunk `next`
  uint32_t slot = 0;
};

// A query whose last chunk ran in some step: where its result row is.
struct Finishing {
  uint64_t tag;
  uint32_t P, Lq;
};

// What one step in flight owns (two of these alternate).
struct StepBuf {
  uint64_t *res = nullptr;      // rows x PI_MAX_L limbs, in finishing order
  size_t res_cap = 0;
  pi_status *res_st = nullptr;  // rows
  size_t res_st_cap = 0;
  HeadSeg *dsegs = nullptr;
  size_t dsegs_cap = 0;
  FinQuery *dfins = nullptr;
  size_t dfins_cap = 0;
  char *pinned = nullptr;       // host staging: tables, then results
  size_t pinned_bytes = 0;
  size_t rhost_off = 0;         // where this step's results land in `pinned`
  hipEvent_t done = nullptr;
  bool busy = false;            // enqueued and not yet harvested
  std::vector<Finishing> fin;
};

uint64_t seg_chunks(const HeadSeg &g) {
  const uint64_t ch = 256ull * g.run;
  return (g.ke - g.kb + ch - 1) / ch;
}

}  // namespace

struct pi_server {
  hipStream_t st = nullptr;
  uint32_t max_active = 0;
  uint32_t cap = 0;                   // slots allocated now
  size_t mem_limit = 0;               // device bytes the slots may take
  uint64_t step_terms = 0;
  unsigned long long *acc = nullptr;  // cap x kSlotCounters, then 2 x kChunkCounters
  StepBuf buf[2];
  int parity = 0;
  int depth = 1;                      // steps left running when pi_server_step returns
  uint32_t in_flight = 0;             // finished queries not yet harvested
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

int grow_pinned(StepBuf &b, size_t need) {
  if (b.pinned_bytes >= need) return PI_OK;
  if (b.pinned) (void)hipHostFree(b.pinned);
  b.pinned = nullptr;
  b.pinned_bytes = 0;
  const size_t n = std::max<size_t>(need, 1 << 16);
  if (hipHostMalloc((void **)&b.pinned, n, hipHostMallocDefault) != hipSuccess) return PI_ENOMEM;
  b.pinned_bytes = n;
  return PI_OK;
}

void release(pi_server *s) {
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->acc) (void)hipFree(s->acc);
  for (StepBuf &b : s->buf) {
    if (b.res) (void)hipFree(b.res);
    if (b.res_st) (void)hipFree(b.res_st);
    if (b.dsegs) (void)hipFree(b.dsegs);
    if (b.dfins) (void)hipFree(b.dfins);
    if (b.pinned) (void)hipHostFree(b.pinned);
    if (b.done) (void)hipEventDestroy(b.done);
  }
}

// The most slots the memory budget and max_active allow.
uint32_t slot_limit(const pi_server *s) {
  return (uint32_t)std::min<uint64_t>(s->max_active, s->mem_limit / kSlotBytes);
}

// Grow the slot pool to `want` slots: a new counter array, the old counters
// copied over once the stream has drained, the old array freed.
int grow_slots(pi_server *s, uint32_t want) {
  if (want <= s->cap) return PI_OK;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return PI_EDEVICE;
  // admission by device memory: never take the last eighth of the device
  const size_t need = (size_t)(want - s->cap) * kSlotBytes;
  if (free_b < need || free_b - need < total_b / 8u) return PI_BUSY;
  unsigned long long *acc = nullptr;
  const size_t words = (size_t)want * kSlotCounters + 2u * kChunkCounters;
  if (hipMalloc((void **)&acc, words * 8u) != hipSuccess) return PI_BUSY;
  if (s->acc) {
    if (hipStreamSynchronize(s->st) != hipSuccess ||
        hipMemcpy(acc, s->acc, (size_t)s->cap * kSlotCounters * 8u, hipMemcpyDeviceToDevice) !=
            hipSuccess) {
      (void)hipFree(acc);
      return PI_EDEVICE;
    }
    (void)hipFree(s->acc);
  }
  s->acc = acc;
  for (uint32_t i = want; i-- > s->cap;) s->free_slots.insert(s->free_slots.begin(), i);
  s->cap = want;
  return PI_OK;
}

// Move a completed step's results to the done list.
int harvest(pi_server *s, StepBuf &b, bool wait) {
  if (!b.busy) return PI_OK;
  if (wait) {
    if (hipEventSynchronize(b.done) != hipSuccess) return PI_EDEVICE;
  } else {
    const hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) return PI_OK;
    if (q != hipSuccess) return PI_EDEVICE;
  }
  const char *rhost = b.pinned + b.rhost_off;
  const char *shost = rhost + b.fin.size() * PI_MAX_L * 8u;
  for (size_t r = 0; r < b.fin.size(); ++r) {
    pi_result res;
    memset(&res, 0, sizeof res);
    pi_status stv;
    memcpy(&stv, shost + r * sizeof(pi_status), sizeof stv);
    res.tag = b.fin[r].tag;
    res.code = stv.code;
    res.P = b.fin[r].P;
    res.nterms = stv.nterms;
    memcpy(res.limbs, rhost + r * PI_MAX_L * 8u, b.fin[r].Lq * 8u);
    s->done.push_back(res);
  }
  s->in_flight -= (uint32_t)b.fin.size();
  b.fin.clear();
  b.busy = false;
  return PI_OK;
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
  pi_server *s = new pi_server();
  s->st = stream;
  s->max_active = max_active;
  s->mem_limit = free_b / 4u;  // default budget: a quarter of what is free now
  s->step_terms = step_terms;
  for (StepBuf &b : s->buf)
    if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
      release(s);
      delete s;
      return PI_EDEVICE;
    }
  const uint32_t first = std::min(kFirstSlots, slot_limit(s));
  if (first == 0 || grow_slots(s, first) != PI_OK) {
    release(s);
    delete s;
    return PI_ENOMEM;
  }
  *out = s;
  return PI_OK;
}

int pi_server_set_memory_limit(pi_server *s, size_t bytes) {
  if (!s) return PI_EINVAL;
  s->mem_limit = bytes;
  return PI_OK;
}

int pi_server_submit(pi_server *s, const pi_query *q, uint64_t tag) {
  if (!s || !q || q->reserved != 0) return PI_EINVAL;
  Active a;
  if (int e = make_plan(q->formula, q->n, q->nbits, q->P, 0x7fu, 0, UINT64_MAX, &a.qp)) return e;
  const uint32_t admitted = (uint32_t)s->active.size() + s->in_flight;
  if (admitted >= slot_limit(s)) return PI_BUSY;
  if (s->free_slots.empty()) {
    // a slot exists only while memory allows: double the pool up to the limit
    if (int e = grow_slots(s, std::min(slot_limit(s), std::max(2u * s->cap, s->cap + 1u))))
      return e;
    if (s->free_slots.empty()) return PI_BUSY;
  }
  a.slot = s->free_slots.back();
  if (int e = hip_err(launch_zero(s->acc + (uint64_t)a.slot * kSlotCounters, kSlotCounters, s->st)))
    return e;
  s->free_slots.pop_back();
  a.tag = tag;
  head_segments(a.qp, a.slot * kSlotCounters, a.segs);
  // A step covers at most step_terms head terms across all queries, so its
  // chunks are kept small enough that every workgroup slot of the launch gets
  // several of them (kStepChunksPerSlot); a long run fits a whole-query launch
  // but leaves a step with a few huge chunks and an idle tail.
  const bool fused = a.qp.Lk <= kFusedMaxL;
  const int grid = fused ? resident_grid_fused() : resident_grid(a.qp.Lk, false);
  const uint64_t step_run = s->step_terms / (256ull * (uint64_t)grid * kStepChunksPerSlot);
  const uint32_t tuned = fused ? run_cap_fused() : run_cap_for(a.qp.Lk);
  const uint32_t run_cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tuned, step_run));
  const uint32_t cap = std::max(pick_run(a.qp.nhead, grid, run_cap), min_run_cap(a.qp.nhead));
  a.nchunks = number_chunks(a.segs, cap, 0);
  s->active.push_back(std::move(a));
  return PI_OK;
}

int pi_server_cancel(pi_server *s, uint64_t tag) {
  if (!s) return PI_EINVAL;
  for (size_t i = 0; i < s->active.size(); ++i)
    if (s->active[i].tag == tag) {
      // chunks of it queued in a step still add into this slot; its next
      // user's clearing kernel is queued behind them on the same stream
      s->free_slots.push_back(s->active[i].slot);
      s->active.erase(s->active.begin() + (std::ptrdiff_t)i);
      return PI_OK;
    }
  return PI_EINVAL;
}

int pi_server_step(pi_server *s, uint32_t *finished) {
  if (!s) return PI_EINVAL;
  if (finished) *finished = 0;
  const size_t before = s->done.size();
  StepBuf &b = s->buf[s->parity];
  StepBuf &prev = s->buf[s->parity ^ 1];
  if (s->active.empty()) {
    // nothing left to plan: wait for what is still on the device
    if (int e = harvest(s, prev, true)) return e;
    if (int e = harvest(s, b, true)) return e;
    if (finished) *finished = (uint32_t)(s->done.size() - before);
    return PI_OK;
  }
  // this buffer's last step (two steps ago) was harvested by the previous call
  if (int e = harvest(s, b, true)) return e;
  // 1. each active query takes chunks worth up to its fair share of terms
  const uint64_t quota = std::max<uint64_t>(1, s->step_terms / s->active.size());
  std::map<int, std::vector<HeadSeg>> segs_by_class;
  std::map<int, uint64_t> chunks_by_class;
  std::vector<size_t> finishing;
  for (size_t i = 0; i < s->active.size(); ++i) {
    Active &a = s->active[i];
    const int Lk = a.qp.Lk <= kFusedMaxL ? 0 : a.qp.Lk;  // launch group, 0: fused
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
  //    their results land in this buffer's rows 0, 1, ... in finishing order
  std::map<int, std::vector<FinQuery>> fins_by_class;
  for (size_t r = 0; r < finishing.size(); ++r) {
    const Active &a = s->active[finishing[r]];
    fins_by_class[a.qp.Lk <= kFusedMaxL ? 0 : a.qp.Lk].push_back(
        fin_query(a.qp, (uint64_t)r * PI_MAX_L, 1u, (uint32_t)r, a.slot * kSlotCounters));
  }
  size_t nsegs = 0, nfins = 0;
  for (auto &kv : segs_by_class) nsegs += kv.second.size();
  for (auto &kv : fins_by_class) nfins += kv.second.size();
  // 3. upload the tables through this buffer's pinned staging
  const size_t tbytes = nsegs * sizeof(HeadSeg) + nfins * sizeof(FinQuery);
  const size_t rbytes = finishing.size() * (PI_MAX_L * 8u + sizeof(pi_status));
  if (int e = grow_device(&b.dsegs, &b.dsegs_cap, nsegs)) return e;
  if (int e = grow_device(&b.dfins, &b.dfins_cap, nfins)) return e;
  if (int e = grow_device(&b.res, &b.res_cap, finishing.size() * PI_MAX_L)) return e;
  if (int e = grow_device(&b.res_st, &b.res_st_cap, finishing.size())) return e;
  if (int e = grow_pinned(b, tbytes + rbytes)) return e;
  size_t so = 0, fo = 0;
  std::map<int, std::pair<size_t, size_t>> seg_at, fin_at;  // class -> (offset, count)
  for (auto &kv : segs_by_class) {
    memcpy(b.pinned + so * sizeof(HeadSeg), kv.second.data(), kv.second.size() * sizeof(HeadSeg));
    seg_at[kv.first] = {so, kv.second.size()};
    so += kv.second.size();
  }
  char *fhost = b.pinned + nsegs * sizeof(HeadSeg);
  for (auto &kv : fins_by_class) {
    memcpy(fhost + fo * sizeof(FinQuery), kv.second.data(), kv.second.size() * sizeof(FinQuery));
    fin_at[kv.first] = {fo, kv.second.size()};
    fo += kv.second.size();
  }
  if (nsegs && hipMemcpyAsync(b.dsegs, b.pinned, nsegs * sizeof(HeadSeg), hipMemcpyHostToDevice,
                              s->st) != hipSuccess)
    return PI_EDEVICE;
  if (nfins && hipMemcpyAsync(b.dfins, fhost, nfins * sizeof(FinQuery), hipMemcpyHostToDevice,
                              s->st) != hipSuccess)
    return PI_EDEVICE;
  // 4. head launches (each with its own chunk counter of this parity, cleared
  //    first), then finalize launches, per launch group: queries of up to
  //    kFusedMaxL limbs together, larger ones per limb class
  unsigned long long *ctr =
      s->acc + (uint64_t)s->cap * kSlotCounters + (uint64_t)s->parity * kChunkCounters;
  if (!seg_at.empty())
    if (int e = hip_err(launch_zero(ctr, kChunkCounters, s->st))) return e;
  int launch = 0;
  for (auto &kv : seg_at) {
    const int Lk = kv.first;
    const uint64_t nch = chunks_by_class[Lk];
    if (!nch) continue;
    const int grid = (int)std::min<uint64_t>(
        nch, (uint64_t)(Lk ? resident_grid(Lk, false) : resident_grid_fused()));
    const HeadSeg *sg = b.dsegs + kv.second.first;
    const int ns = (int)kv.second.second;
    const hipError_t he = Lk ? launch_head_ptr(Lk, sg, ns, nch, grid, s->acc, ctr + launch, s->st)
                             : launch_head_fused(sg, ns, nch, grid, s->acc, ctr + launch, s->st);
    ++launch;
    if (int e = hip_err(he)) return e;
  }
  FinQuery none;
  memset(&none, 0, sizeof none);
  for (auto &kv : fin_at) {
    const FinQuery *fq = b.dfins + kv.second.first;
    const int nf = (int)kv.second.second;
    const hipError_t fe =
        kv.first ? launch_finalize(kv.first, none, fq, nf, s->acc, b.res, b.res_st, s->st)
                 : launch_finalize_fused(fq, nf, s->acc, b.res, b.res_st, s->st);
    if (int e = hip_err(fe)) return e;
  }
  // 5. the finished rows come home after the step; the event marks the end
  b.rhost_off = tbytes;
  char *rhost = b.pinned + tbytes;
  char *shost = rhost + finishing.size() * PI_MAX_L * 8u;
  if (!finishing.empty()) {
    if (hipMemcpyAsync(rhost, b.res, finishing.size() * PI_MAX_L * 8u, hipMemcpyDeviceToHost,
                       s->st) != hipSuccess ||
        hipMemcpyAsync(shost, b.res_st, finishing.size() * sizeof(pi_status),
                       hipMemcpyDeviceToHost, s->st) != hipSuccess)
      return PI_EDEVICE;
  }
  if (hipEventRecord(b.done, s->st) != hipSuccess) return PI_EDEVICE;
  b.busy = true;
  // 6. retire the finishing queries now: their rows belong to this buffer,
  //    and a slot's next user clears it with a kernel queued behind this step
  std::vector<bool> gone(s->active.size(), false);
  for (size_t i : finishing) {
    const Active &a = s->active[i];
    b.fin.push_back({a.tag, a.qp.P, a.qp.Lq});
    gone[i] = true;
    s->free_slots.push_back(a.slot);
  }
  s->in_flight += (uint32_t)finishing.size();
  size_t w = 0;
  for (size_t i = 0; i < s->active.size(); ++i)
    if (!gone[i]) {
      if (w != i) s->active[w] = std::move(s->active[i]);
      ++w;
    }
  s->active.resize(w);
  s->parity ^= 1;
  // 7. wait for the previous step (this one runs on) and deliver its results;
  //    unpipelined, wait for this one too
  if (int e = harvest(s, prev, true)) return e;
  if (s->depth == 0)
    if (int e = harvest(s, b, true)) return e;
  if (finished) *finished = (uint32_t)(s->done.size() - before);
  return PI_OK;
}

int pi_server_set_pipeline(pi_server *s, int depth) {
  if (!s || depth < 0 || depth > 1) return PI_EINVAL;
  s->depth = depth;
  return PI_OK;
}

int pi_server_poll(pi_server *s, pi_result *out, uint32_t max, uint32_t *count) {
  if (!s || !count || (max && !out)) return PI_EINVAL;
  for (StepBuf &b : s->buf)
    if (int e = harvest(s, b, false)) return e;
  uint32_t n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *count = n;
  return PI_OK;
}

uint32_t pi_server_active(const pi_server *s) {
  return s ? (uint32_t)s->active.size() + s->in_flight : 0;
}

uint32_t pi_server_capacity(const pi_server *s) { return s ? slot_limit(s) : 0; }

void pi_server_destroy(pi_server *s) {
  if (!s) return;
  release(s);
  delete s;
}

}  // extern "C"
