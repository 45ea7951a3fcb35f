// The continuous-batching server's bookkeeping on the CPU
// (tests/test_server_model.py). server.cpp and abi.cpp run unchanged on
// tests/fake_hip.cpp (host memory; stream work deferred until the host waits,
// as on a device) with the stand-ins below for the kernels. The stand-ins check what the kernels rely on and do
// a countable version of their work:
//  * a head launch finds its chunk counter cleared, and its segments are
//    numbered from chunk 0 without gaps up to the launch's chunk count;
//  * it adds each segment's index count to its query's first counter and
//    records the segment's index range against those counters; two launches
//    never cover the same index of one query;
//  * a finalize finds, for every series of its query, ranges that tile the
//    head range [0, first tail index) exactly, and a count equal to the
//    query's head count; it writes that count and d = n - 1 to the result row.
// Clearing a query's counters forgets its ranges; a copy of the counters to a
// new array (the slot pool growing) moves them.
// The program streams seeded queries through servers of several shapes, in
// both pipeline modes, and checks that every query comes back once, under its
// own tag, with its own head count; whole queries through the single-query,
// allocation-free and batch front ends get the same checks.
#include <inttypes.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <memory>
#include <vector>

#include "pibbp.h"
#include "plan.h"

extern void (*fake_hip_on_copy)(void *dst, const void *src, size_t n);
extern void (*fake_hip_on_free)(void *p, size_t n);
extern size_t fake_hip_free_bytes;
void fake_hip_enqueue(std::function<void()> f);

namespace {

int g_fail = 0;
#define CHECK(c, ...)                \
  do {                               \
    if (!(c)) {                      \
      if (g_fail < 20) {             \
        fprintf(stderr, __VA_ARGS__); \
        fputc('\n', stderr);         \
      }                              \
      ++g_fail;                      \
    }                                \
  } while (0)

using Ranges = std::map<int, std::vector<std::pair<uint64_t, uint64_t>>>;
std::map<uintptr_t, Ranges> g_cover;  // query counters' address -> series -> index ranges
uint64_t g_head_launches = 0, g_fin_launches = 0, g_finalized = 0;

void forget(uintptr_t p, size_t n) {
  g_cover.erase(g_cover.lower_bound(p), g_cover.lower_bound(p + n));
}

// A copy replaces whatever the destination held; freed memory holds nothing.
void on_copy(void *dst, const void *src, size_t n) {
  const uintptr_t s = (uintptr_t)src, d = (uintptr_t)dst;
  auto lo = g_cover.lower_bound(s), hi = g_cover.lower_bound(s + n);
  std::vector<std::pair<uintptr_t, Ranges>> moved;
  for (auto it = lo; it != hi; ++it) moved.emplace_back(it->first - s + d, std::move(it->second));
  g_cover.erase(lo, hi);
  forget(d, n);
  for (auto &m : moved) g_cover[m.first] = std::move(m.second);
}

void on_free(void *p, size_t n) { forget((uintptr_t)p, n); }

void head(const pibbp::HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
          unsigned long long *acc, unsigned long long *ctr) {
  CHECK(*ctr == 0, "head launch: chunk counter not cleared");
  *ctr = nchunks;
  CHECK(grid >= 1 && (uint64_t)grid <= nchunks, "head launch: grid %d for %" PRIu64 " chunks",
        grid, nchunks);
  uint64_t c = 0;
  for (int i = 0; i < nseg; ++i) {
    const pibbp::HeadSeg &g = segs[i];
    CHECK(g.chunk0 == c, "segment %d numbered from %" PRIu64 ", expected %" PRIu64, i,
          (uint64_t)g.chunk0, c);
    CHECK(g.ke > g.kb && g.run >= 1, "empty segment or run 0");
    if (g.run >= 1) c += (g.ke - g.kb + 256ull * g.run - 1) / (256ull * g.run);
    auto &iv = g_cover[(uintptr_t)(acc + g.acc_off)][g.j];
    for (auto &p : iv)
      CHECK(g.ke <= p.first || p.second <= g.kb,
            "series %d: [%" PRIu64 ", %" PRIu64 ") launched twice", (int)g.j, (uint64_t)g.kb,
            (uint64_t)g.ke);
    iv.emplace_back(g.kb, g.ke);
    acc[g.acc_off] += g.ke - g.kb;
  }
  CHECK(c == nchunks, "segments hold %" PRIu64 " chunks, launch says %" PRIu64, c, nchunks);
  ++g_head_launches;
}

void finalize(const pibbp::FinQuery *qs, int nq, const unsigned long long *acc, uint64_t *out,
              pi_status *st) {
  for (int i = 0; i < nq; ++i) {
    const pibbp::FinQuery &q = qs[i];
    Ranges &r = g_cover[(uintptr_t)(acc + q.acc_off)];
    for (int j = 0; j < 7; ++j) {
      auto iv = r[j];
      std::sort(iv.begin(), iv.end());
      uint64_t at = 0;
      for (auto &p : iv) {
        CHECK(p.first == at, "series %d: gap or overlap at %" PRIu64, j, at);
        at = p.second;
      }
      CHECK(at == q.tk0[j], "series %d: head covered to %" PRIu64 ", first tail index %" PRIu64,
            j, at, (uint64_t)q.tk0[j]);
    }
    CHECK(acc[q.acc_off] == q.nhead, "head count %llu, plan %" PRIu64, acc[q.acc_off],
          (uint64_t)q.nhead);
    out[q.out_off] = acc[q.acc_off];
    if (q.Lq >= 2) out[q.out_off + 1] = q.d;  // a batch packs rows of Lq limbs
    if (q.want_status) {
      st[q.status_idx].code = PI_OK;
      st[q.status_idx].reserved = 0;
      st[q.status_idx].nterms = q.nhead;
    }
    ++g_finalized;
  }
  ++g_fin_launches;
}

}  // namespace

namespace pibbp {
// Each stand-in runs when the stream reaches it (fake_hip_enqueue), reading
// device memory then; arguments passed by value are copied now, as a kernel
// launch copies its arguments.
hipError_t launch_zero(unsigned long long *p, uint64_t n, hipStream_t) {
  fake_hip_enqueue([=] {
    memset(p, 0, n * 8);
    g_cover.erase(g_cover.lower_bound((uintptr_t)p), g_cover.lower_bound((uintptr_t)(p + n)));
  });
  return hipSuccess;
}
hipError_t launch_head_ptr(int, const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                           unsigned long long *acc, unsigned long long *ctr, hipStream_t) {
  fake_hip_enqueue([=] { head(segs, nseg, nchunks, grid, acc, ctr); });
  return hipSuccess;
}
hipError_t launch_head_fused(const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                             unsigned long long *acc, unsigned long long *ctr, hipStream_t) {
  fake_hip_enqueue([=] {
    for (int i = 0; i < nseg; ++i)
      CHECK((segs[i].P + 63u) / 64u <= (uint32_t)kFusedMaxL, "a wide query in the fused launch");
    head(segs, nseg, nchunks, grid, acc, ctr);
  });
  return hipSuccess;
}
hipError_t launch_head_args(int, const HeadSegTable &tab, uint64_t nchunks, int grid,
                            unsigned long long *acc, unsigned long long *ctr, hipStream_t) {
  auto t = std::make_shared<HeadSegTable>(tab);
  fake_hip_enqueue([=] { head(t->s, t->n, nchunks, grid, acc, ctr); });
  return hipSuccess;
}
hipError_t launch_finalize(int, const FinQuery &single, const FinQuery *qs, int nq,
                           const unsigned long long *acc, uint64_t *out, pi_status *status,
                           hipStream_t) {
  const FinQuery one = single;
  fake_hip_enqueue([=] { finalize(qs ? qs : &one, qs ? nq : 1, acc, out, status); });
  return hipSuccess;
}
hipError_t launch_finalize_fused(const FinQuery *qs, int nq, const unsigned long long *acc,
                                 uint64_t *out, pi_status *status, hipStream_t) {
  fake_hip_enqueue([=] { finalize(qs, nq, acc, out, status); });
  return hipSuccess;
}
hipError_t launch_combine(const uint64_t *, int, int, uint32_t, uint32_t, uint64_t, uint32_t,
                          uint64_t *, pi_status *, hipStream_t) {
  return hipErrorNotSupported;
}
int head_occupancy_fused() { return 6; }
int head_occupancy(int Lk, bool) { return Lk <= 8 ? 7 : 4; }
unsigned long long g_static[64];
hipError_t static_scratch(unsigned long long **ptr, uint32_t *words) {
  memset(g_static, 0xA5, sizeof g_static);  // holds whatever the last call left
  *ptr = g_static;
  *words = 64;
  return hipSuccess;
}
}  // namespace pibbp

namespace {

uint64_t g_state = 0x13198a2e03707344ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
uint64_t below(uint64_t n) { return n ? next_u64() % n : 0; }

struct Query {
  pi_query q;
  bool back = false;
  bool cancelled = false;
};

// cancel_one_in: after a step, with probability 1/cancel_one_in, withdraw a
// random first-submission query still out and submit it again under a new
// tag (at most count / 5 times, so that the stream ends). mem_limit 1 means a
// budget of exactly max_active slots, so that a slot a withdrawal failed to
// free would stall the stream.
void scenario(const char *name, uint32_t max_active, uint64_t step_terms, size_t mem_limit,
              int depth, int count, int max_bits, int cancel_one_in = 0) {
  std::vector<Query> qs(count);
  for (Query &x : qs) {
    memset(&x.q, 0, sizeof x.q);
    x.q.formula = (int32_t)below(2);
    x.q.n = 1 + below(1ull << (1 + below(max_bits)));      // log-uniform positions
    x.q.nbits = 1 + (uint32_t)below(256);
    x.q.P = x.q.nbits + (uint32_t)below(PI_MAX_P - x.q.nbits + 1);
  }
  pi_server *s = nullptr;
  int rc = pi_server_create(max_active, step_terms, nullptr, &s);
  CHECK(rc == PI_OK && s, "%s: create -> %d", name, rc);
  if (!s) return;
  if (mem_limit == 1) {  // the bytes of one slot, from the capacity a large budget buys
    pi_server *probe = nullptr;
    CHECK(pi_server_create(1u << 30, step_terms, nullptr, &probe) == PI_OK, "probe");
    CHECK(pi_server_set_memory_limit(probe, (size_t)1 << 32) == PI_OK, "probe limit");
    const size_t slot = ((size_t)1 << 32) / pi_server_capacity(probe);
    pi_server_destroy(probe);
    mem_limit = max_active * slot + slot / 2;
  }
  if (mem_limit) CHECK(pi_server_set_memory_limit(s, mem_limit) == PI_OK, "memory limit");
  CHECK(pi_server_set_pipeline(s, depth) == PI_OK, "pipeline");
  const uint32_t cap = pi_server_capacity(s);
  size_t next = 0, back = 0, cancelled = 0, refused = 0;
  uint64_t steps = 0;
  uint32_t most = 0;
  std::vector<pi_result> res(64);
  while (back + cancelled < qs.size()) {
    while (next < qs.size()) {
      rc = pi_server_submit(s, &qs[next].q, next);
      if (rc == PI_BUSY) break;
      CHECK(rc == PI_OK, "%s: submit %zu -> %d", name, next, rc);
      ++next;
    }
    most = std::max(most, pi_server_active(s));
    CHECK(pi_server_active(s) <= cap, "%s: %u admitted over capacity %u", name,
          pi_server_active(s), cap);
    uint32_t fin = 0;
    rc = pi_server_step(s, &fin);
    CHECK(rc == PI_OK, "%s: step -> %d", name, rc);
    ++steps;
    uint32_t got = 0;
    do {
      CHECK(pi_server_poll(s, res.data(), (uint32_t)res.size(), &got) == PI_OK, "poll");
      for (uint32_t i = 0; i < got; ++i) {
        const pi_result &r = res[i];
        CHECK(r.tag < qs.size() && !qs[r.tag].back && !qs[r.tag].cancelled,
              "%s: tag %" PRIu64 " unknown, repeated or withdrawn", name, r.tag);
        if (r.tag >= qs.size() || qs[r.tag].back || qs[r.tag].cancelled) continue;
        Query &x = qs[r.tag];
        x.back = true;
        ++back;
        const uint64_t want = pi_head_terms(x.q.formula, x.q.n);
        // the row's second limb (d) comes back only when the query has two limbs
        CHECK(r.code == PI_OK && r.P == x.q.P && r.limbs[0] == want && r.nterms == want &&
                  (x.q.P <= 64 || r.limbs[1] == x.q.n - 1),
              "%s: tag %" PRIu64 ": code %d P %u count %" PRIu64 "/%" PRIu64 " (want %" PRIu64
              ") d %" PRIu64,
              name, r.tag, r.code, r.P, (uint64_t)r.limbs[0], (uint64_t)r.nterms, want,
              (uint64_t)r.limbs[1]);
      }
    } while (got == res.size());
    if (cancel_one_in && below(cancel_one_in) == 0 && cancelled < (size_t)count / 5) {
      std::vector<size_t> out;
      for (size_t t = 0; t < std::min(next, (size_t)count); ++t)
        if (!qs[t].back && !qs[t].cancelled) out.push_back(t);
      if (!out.empty()) {
        const size_t t = out[below(out.size())];
        rc = pi_server_cancel(s, t);
        CHECK(rc == PI_OK || rc == PI_EINVAL, "%s: cancel -> %d", name, rc);
        if (rc == PI_OK) {  // withdrawn: submit the same query again later
          qs[t].cancelled = true;
          ++cancelled;
          Query again;
          again.q = qs[t].q;
          qs.push_back(again);
        } else {
          ++refused;  // its last chunks already ran: its result is on the way
        }
      }
      CHECK(pi_server_cancel(s, 1ull << 40) == PI_EINVAL, "%s: unknown tag cancelled", name);
    }
    if (steps > 200000) {
      CHECK(false, "%s: no progress", name);
      break;
    }
  }
  CHECK(pi_server_active(s) == 0, "%s: %u still active", name, pi_server_active(s));
  // every slot came back: a full burst is admitted at once, and finishes
  pi_query small;
  memset(&small, 0, sizeof small);
  small.formula = PI_BELLARD;
  small.n = 1000;
  small.nbits = 32;
  small.P = 96;
  for (uint32_t i = 0; i < cap; ++i) {
    rc = pi_server_submit(s, &small, 1ull << 41);
    CHECK(rc == PI_OK, "%s: slot %u of %u not free after the stream (%d)", name, i, cap, rc);
    if (rc != PI_OK) break;
  }
  for (int i = 0; i < 1000 && pi_server_active(s); ++i) {
    uint32_t got = 0;
    CHECK(pi_server_step(s, nullptr) == PI_OK, "step");
    do CHECK(pi_server_poll(s, res.data(), (uint32_t)res.size(), &got) == PI_OK, "poll");
    while (got == res.size());
  }
  CHECK(pi_server_active(s) == 0, "%s: the burst did not finish", name);
  pi_server_destroy(s);
  if (cancel_one_in) CHECK(cancelled > 0, "%s: nothing was withdrawn", name);
  printf("%s: depth %d, capacity %u, most admitted %u, %" PRIu64 " steps, %zu queries back, %zu "
         "withdrawn and submitted again, %zu cancels refused\n",
         name, depth, cap, most, steps, back, cancelled, refused);
}

}  // namespace

// Whole queries through the other front ends: one call each (pi_extract_ex,
// pi_extract_noalloc), a batch (pi_extract_batch, and a plan launched three
// times). Each query's row must hold its own head count (and d), and its
// status that count.
void front_ends(int count) {
  std::vector<pi_query> q(count);
  uint64_t rows = 0;
  for (pi_query &x : q) {
    memset(&x, 0, sizeof x);
    x.formula = (int32_t)below(2);
    x.n = 1 + below(1ull << (1 + below(34)));
    x.nbits = 1 + (uint32_t)below(256);
    x.P = x.nbits + (uint32_t)below(PI_MAX_P - x.nbits + 1);
    x.out_offset = rows;
    rows += (x.P + 63u) / 64u;
  }
  auto check = [&](const char *what, int i, const uint64_t *row, const pi_status &st) {
    const pi_query &x = q[i];
    const uint64_t want = pi_head_terms(x.formula, x.n);
    CHECK(row[0] == want && (x.P <= 64 || row[1] == x.n - 1) && st.code == PI_OK &&
              st.nterms == want,
          "%s: query %d: count %" PRIu64 " (want %" PRIu64 "), status %d/%" PRIu64, what, i,
          (uint64_t)row[0], want, st.code, (uint64_t)st.nterms);
  };
  std::vector<uint64_t> out(rows + pibbp::PI_MAX_L);
  std::vector<pi_status> st(count);
  for (int i = 0; i < count; ++i) {
    uint64_t row[pibbp::PI_MAX_L] = {};
    pi_status one = {};
    int rc = pi_extract_ex(q[i].formula, q[i].n, q[i].nbits, q[i].P, row, &one, nullptr);
    CHECK(rc == PI_OK, "extract_ex -> %d", rc);
    (void)hipStreamSynchronize(nullptr);  // results are ready when the stream is
    check("extract_ex", i, row, one);
    memset(row, 0, sizeof row);
    memset(&one, 0, sizeof one);
    rc = pi_extract_noalloc(q[i].formula, q[i].n, q[i].nbits, q[i].P, row, &one, nullptr);
    CHECK(rc == PI_OK, "extract_noalloc -> %d", rc);
    (void)hipStreamSynchronize(nullptr);
    check("extract_noalloc", i, row, one);
  }
  int rc = pi_extract_batch(q.data(), count, out.data(), st.data(), nullptr, 0, nullptr);
  CHECK(rc == PI_OK, "extract_batch -> %d", rc);
  (void)hipStreamSynchronize(nullptr);
  for (int i = 0; i < count; ++i) check("extract_batch", i, &out[q[i].out_offset], st[i]);
  // two batches back to back, nothing waited for in between: the second
  // must not rewrite the staging the first one's table upload still reads
  {
    const int half = count / 2;
    std::vector<uint64_t> out2(rows + pibbp::PI_MAX_L);
    std::vector<pi_status> st2(count);
    std::vector<pi_query> second(q.begin() + half, q.end());
    std::fill(out.begin(), out.end(), 0);
    memset(st.data(), 0, st.size() * sizeof(pi_status));
    rc = pi_extract_batch(q.data(), half, out.data(), st.data(), nullptr, 0, nullptr);
    CHECK(rc == PI_OK, "first batch -> %d", rc);
    rc = pi_extract_batch(second.data(), count - half, out2.data(), st2.data(), nullptr, 0,
                          nullptr);
    CHECK(rc == PI_OK, "second batch -> %d", rc);
    (void)hipStreamSynchronize(nullptr);
    for (int i = 0; i < half; ++i) check("first batch", i, &out[q[i].out_offset], st[i]);
    for (int i = half; i < count; ++i)
      check("second batch", i, &out2[q[i].out_offset], st2[i - half]);
  }
  pi_batch *plan = nullptr;
  rc = pi_batch_create(q.data(), count, out.data(), st.data(), &plan);
  CHECK(rc == PI_OK && plan, "batch_create -> %d", rc);
  for (int rep = 0; plan && rep < 3; ++rep) {
    std::fill(out.begin(), out.end(), 0);
    memset(st.data(), 0, st.size() * sizeof(pi_status));
    rc = pi_batch_launch(plan, nullptr);
    CHECK(rc == PI_OK, "batch_launch -> %d", rc);
    (void)hipStreamSynchronize(nullptr);
    for (int i = 0; i < count; ++i) check("batch plan", i, &out[q[i].out_offset], st[i]);
  }
  pi_batch_destroy(plan);
  pi_shutdown();  // the per-stream scratch and staging the library keeps
  printf("front ends: %d queries\n", count);
}

// The memory budget cut below what is admitted, mid-stream: nothing more is
// admitted until the active queries fit it, and every result still comes back.
void shrinking_budget(int depth) {
  pi_server *s = nullptr;
  CHECK(pi_server_create(64, 1ull << 24, nullptr, &s) == PI_OK, "create");
  CHECK(pi_server_set_pipeline(s, depth) == PI_OK, "pipeline");
  size_t slot = 0;  // the bytes of one slot, from the capacity a large budget buys
  {
    pi_server *probe = nullptr;
    CHECK(pi_server_create(1u << 30, 1ull << 24, nullptr, &probe) == PI_OK, "probe");
    CHECK(pi_server_set_memory_limit(probe, (size_t)1 << 32) == PI_OK, "probe limit");
    slot = ((size_t)1 << 32) / pi_server_capacity(probe);
    pi_server_destroy(probe);
  }
  std::vector<pi_query> q(120);
  for (pi_query &x : q) {
    memset(&x, 0, sizeof x);
    x.formula = (int32_t)below(2);
    x.n = 1 + below(1ull << (1 + below(30)));
    x.nbits = 64;
    x.P = 64 + (uint32_t)below(PI_MAX_P - 63);
  }
  CHECK(pi_server_set_memory_limit(s, 64 * slot + slot / 2) == PI_OK, "limit");
  size_t next = 0, back = 0, steps = 0, refused = 0;
  std::vector<bool> seen(q.size(), false);
  std::vector<pi_result> res(64);
  while (back < q.size() && steps < 200000) {
    while (next < q.size()) {
      const uint32_t before = pi_server_active(s);
      const int rc = pi_server_submit(s, &q[next], next);
      if (rc == PI_BUSY) {
        CHECK(before >= pi_server_capacity(s) || before >= 64, "busy with room: %u of %u", before,
              pi_server_capacity(s));
        ++refused;
        break;
      }
      CHECK(rc == PI_OK && before < pi_server_capacity(s), "admitted %u over capacity %u", before,
            pi_server_capacity(s));
      ++next;
    }
    CHECK(pi_server_step(s, nullptr) == PI_OK, "step");
    if (++steps == 3)  // cut the budget to 10 slots while about 64 queries are in
      CHECK(pi_server_set_memory_limit(s, 10 * slot + slot / 2) == PI_OK &&
                pi_server_capacity(s) == 10,
            "cut budget");
    uint32_t got = 0;
    do {
      CHECK(pi_server_poll(s, res.data(), (uint32_t)res.size(), &got) == PI_OK, "poll");
      for (uint32_t i = 0; i < got; ++i) {
        const pi_result &r = res[i];
        CHECK(r.tag < q.size() && !seen[r.tag], "tag %" PRIu64 " unknown or repeated", r.tag);
        if (r.tag >= q.size() || seen[r.tag]) continue;
        seen[r.tag] = true;
        ++back;
        const uint64_t want = pi_head_terms(q[r.tag].formula, q[r.tag].n);
        CHECK(r.code == PI_OK && r.limbs[0] == want, "shrinking budget: tag %" PRIu64, r.tag);
      }
    } while (got == res.size());
  }
  CHECK(back == q.size(), "shrinking budget: %zu of %zu back", back, q.size());
  pi_server_destroy(s);
  printf("shrinking budget: depth %d, %zu steps, %zu queries back, %zu submissions refused\n",
         depth, steps, back, refused);
}

int main() {
  fake_hip_on_copy = on_copy;
  fake_hip_on_free = on_free;
  front_ends(300);
  for (int depth = 1; depth >= 0; --depth) {
    scenario("small steps", 64, 1ull << 22, 0, depth, 200, 30);
    scenario("pool growth", 400, 1ull << 30, 0, depth, 1200, 34);
    scenario("memory limit", 1000, 1ull << 28, 40 * 4096, depth, 500, 32);
    scenario("one at a time", 1, 1ull << 30, 0, depth, 40, 36);
    scenario("cancel and resubmit", 64, 1ull << 26, 1, depth, 300, 32, 3);
    shrinking_budget(depth);
  }
  // a budget below one slot admits nothing: creation fails cleanly
  const size_t before = fake_hip_free_bytes;
  fake_hip_free_bytes = 1 << 20;
  pi_server *s = nullptr;
  const int rc = pi_server_create(8, 1 << 20, nullptr, &s);
  CHECK(rc == PI_ENOMEM && !s, "create with no memory -> %d", rc);
  fake_hip_free_bytes = before;
  printf("head launches %" PRIu64 ", finalize launches %" PRIu64 ", queries finalized %" PRIu64
         ", failures %d\n",
         g_head_launches, g_fin_launches, g_finalized, g_fail);
  return g_fail ? 1 : 0;
}
