// A host-only test program for the library's planning code (abi.cpp, server.cpp)
// built with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_host_sanitized.py). The kernels are not linked in:
// every launcher below is a stand-in that reports "no device" and counts its
// calls, and the HIP runtime finds no GPU on the build host, so each entry
// point runs its argument checks and planning and stops at its first device
// call. The program prints every result as text; the test compares the
// sanitized build with a plain one.
#include <inttypes.h>
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "pibbp.h"
#include "plan.h"

namespace pibbp {
static int g_launches = 0;
hipError_t launch_head_args(int, const HeadSegTable &, uint64_t, int, unsigned long long *,
                            unsigned long long *, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
hipError_t launch_head_ptr(int, const HeadSeg *, int, uint64_t, int, unsigned long long *,
                           unsigned long long *, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
hipError_t launch_finalize(int, const FinQuery &, const FinQuery *, int,
                           const unsigned long long *, uint64_t *, pi_status *, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
hipError_t launch_zero(unsigned long long *, uint64_t, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
hipError_t launch_head_fused(const HeadSeg *, int, uint64_t, int, unsigned long long *,
                             unsigned long long *, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
hipError_t launch_finalize_fused(const FinQuery *, int, const unsigned long long *, uint64_t *,
                                 pi_status *, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
hipError_t launch_combine(const uint64_t *, int, int, uint32_t, uint32_t, uint64_t, uint32_t,
                          uint64_t *, pi_status *, hipStream_t) {
  ++g_launches;
  return hipErrorNoDevice;
}
int head_occupancy_fused() { return 1; }
int head_occupancy(int, bool) { return 1; }
hipError_t static_scratch(unsigned long long **, uint32_t *) { return hipErrorNoDevice; }
}  // namespace pibbp

namespace {

uint64_t g_state = 0x243f6a8885a308d3ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
uint64_t below(uint64_t n) { return n ? next_u64() % n : 0; }

uint64_t random_n() {
  static const uint64_t big[] = {1, 2, 3, 9, 10, 1000001, 1000000000001ull,
                                 2000000000000000ull - 3, 2000000000000000ull,
                                 (1ull << 62) - PI_MAX_P - 65, (1ull << 62) - PI_MAX_P - 64};
  if (below(3) == 0) return big[below(sizeof big / sizeof big[0])];
  return 1 + below(1ull << below(52));
}

void plan_one(int arith, int formula, uint64_t n, uint32_t P, uint64_t k0, uint64_t k1,
              uint32_t mask) {
  pi_segment segs[64];
  int count = -1;
  const int rc = pi_plan_head(formula, mask, n, k0, k1, P, segs, 64, &count);
  printf("plan %d %d %" PRIu64 " %u %" PRIu64 " %" PRIu64 " %u -> %d %d\n", arith, formula, n,
         P, k0, k1, mask, rc, count);
  if (rc != PI_OK) return;
  for (int i = 0; i < count; ++i)
    printf("  seg %u %u %u %u %" PRIu64 " %" PRIu64 " %" PRIu64 "\n", segs[i].j, segs[i].cls,
           segs[i].run, segs[i].pre, segs[i].kb, segs[i].ke, segs[i].nchunks);
}

}  // namespace

int main() {
  // head term counts
  for (int f = 0; f < 3; ++f)
    for (int i = 0; i < 40; ++i) {
      const uint64_t n = random_n();
      printf("terms %d %" PRIu64 " %" PRIu64 "\n", f, n, pi_head_terms(f, n));
    }

  // the planner, both arithmetic modes, whole queries and slices
  for (int arith = 0; arith < 2; ++arith) {
    printf("set_arith %d -> %d\n", arith, pi_set_arith(arith));
    for (int i = 0; i < 400; ++i) {
      const int formula = (int)below(2);
      const uint64_t n = random_n();
      const uint32_t P = 1 + (uint32_t)below(below(4) == 0 ? 1200 : PI_MAX_P);
      uint64_t k0 = 0, k1 = UINT64_MAX;
      if (below(2)) {
        k0 = below(n / 4 + 10);
        k1 = below(2) ? k0 + below(1ull << below(40)) : UINT64_MAX;
      }
      const uint32_t mask = below(3) ? 0x7fu : (uint32_t)below(128);
      plan_one(arith, formula, n, P, k0, k1, mask);
    }
  }
  printf("set_arith %d -> %d\n", PI_ARITH_FAST, pi_set_arith(PI_ARITH_FAST));

  // batches: workspace sizes, then creation and extraction up to the first device call
  for (int b = 0; b < 60; ++b) {
    std::vector<pi_query> q(1 + below(b < 50 ? 40 : 4000));
    uint64_t off = 0;
    for (pi_query &x : q) {
      x.formula = (int32_t)below(2);
      x.n = below(100) == 0 ? random_n() : 1 + below(1ull << below(48));
      x.nbits = 1 + (uint32_t)below(256);
      x.P = x.nbits + (uint32_t)below(PI_MAX_P - x.nbits + 1);
      x.reserved = below(2000) == 0 ? 1u : 0u;
      x.out_offset = off;
      off += (x.P + 63u) / 64u;
    }
    const int count = (int)q.size();
    printf("workspace %d %zu\n", count, pi_workspace_size(q.data(), count));
    uint64_t *fake = reinterpret_cast<uint64_t *>(uintptr_t{4096});  // never dereferenced
    pi_batch *plan = nullptr;
    printf("batch_create %d -> %d\n", count, pi_batch_create(q.data(), count, fake, nullptr, &plan));
    if (plan) pi_batch_destroy(plan);
    printf("extract_batch %d -> %d\n", count,
           pi_extract_batch(q.data(), count, fake, nullptr, nullptr, 0, nullptr));
  }

  // single calls: validation, then the first device call
  for (int i = 0; i < 200; ++i) {
    const int formula = (int)below(3);
    const uint64_t n = random_n() - (below(10) == 0 ? 1 : 0);
    const uint32_t nbits = (uint32_t)below(300);
    const uint32_t P = (uint32_t)below(1200);
    uint64_t *fake = below(10) == 0 ? nullptr : reinterpret_cast<uint64_t *>(uintptr_t{4096});
    printf("extract_ex %d %" PRIu64 " %u %u -> %d\n", formula, n, nbits, P,
           pi_extract_ex(formula, n, nbits, P, fake, nullptr, nullptr));
    printf("extract_noalloc %d %" PRIu64 " %u %u -> %d\n", formula, n, nbits, P,
           pi_extract_noalloc(formula, n, nbits, P, fake, nullptr, nullptr));
    printf("extract %d %" PRIu64 " %u -> %d\n", formula, n, nbits,
           pi_extract(formula, n, nbits, fake, nullptr));
    const int term = (int)below(40);
    const uint64_t k0 = below(1000), k1 = k0 + below(1000);
    printf("sum_slice %d %" PRIu64 " %" PRIu64 " %" PRIu64 " %u -> %d %d\n", term, n, k0, k1, P,
           pi_sum_slice(term, n, k0, k1, P, fake, nullptr),
           pi_sum_slice_ex(term, n, k0, k1, P, fake, nullptr, nullptr));
    printf("combine %u %u -> %d\n", P, nbits,
           pi_combine(nullptr, 0, P, nbits, 7, 100, below(2) ? fake : nullptr, nullptr, nullptr));
  }

  // tuning and error strings
  for (int L = -3; L <= pibbp::PI_MAX_L + 1; ++L) {
    uint32_t wg = 0, cap = 0;
    const int s = pi_set_tuning(L, (uint32_t)below(70), (uint32_t)below(5000));
    const int g = pi_get_tuning(L, &wg, &cap);
    printf("tuning %d -> %d %d %u %u\n", L, s, g, wg, cap);
  }
  for (int c = -6; c <= 2; ++c) printf("strerror %d %s\n", c, pi_strerror(c));

  // the server stops at its first device call
  pi_server *srv = nullptr;
  printf("server_create -> %d\n", pi_server_create(16, 1u << 20, nullptr, &srv));
  if (srv) pi_server_destroy(srv);
  printf("server_create bad -> %d\n", pi_server_create(0, 1u << 20, nullptr, &srv));
  pi_shutdown();
  printf("launches %d\n", pibbp::g_launches);
  return 0;
}
