// Work descriptors passed from the host planner to the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pibbp.h"

namespace pibbp {

constexpr int PI_MAX_L = 17;          // ceil(PI_MAX_P / 64)
constexpr int kMaxArgSegs = 56;       // 7 series x 8 modulus ranges

// A range [kb, ke) of head indices (E >= 0) of series j of one query, all of
// one modulus class; its chunks are numbered chunk0, chunk0 + 1, ...
struct HeadSeg {
  uint64_t kb, ke;
  uint64_t chunk0;
  uint64_t d;          // n - 1
  uint32_t P;
  uint32_t acc_off;    // the query's carry-save counters: acc + acc_off
  uint32_t run;        // indices per lane per chunk; a chunk is 256 * run indices
  uint8_t formula, j;
  uint8_t cls;         // arithmetic by modulus: R = 2^32 Montgomery 22 (M < 2^22),
                       // 27 (< 2^27), 29 (< 2^29); binary64 33 (< 2^33), 42 (< 2^42),
                       // 48 (< 2^48), 51 (< 2^51); 64: R = 2^62 Montgomery (M < 2^54)
  uint8_t pre;         // class 62: exponent bits taken into the ladder's start value
};
static_assert(sizeof(HeadSeg) == 48, "HeadSeg layout");

// Segments of a single query, passed by value as a kernel argument.
struct HeadSegTable {
  HeadSeg s[kMaxArgSegs];
  int32_t n;
  int32_t pad;
};

// What the finalize kernel needs for one query: the tail index range of each
// series, the head term count, and where to write.
struct FinQuery {
  uint64_t d;
  uint64_t nhead;      // head indices summed (N before the tail)
  uint64_t out_off;    // in limbs
  uint64_t tk0[7], tk1[7];
  uint32_t formula, P, w, Lq;
  uint32_t want_status;  // 0: none, 1: certify, 2: report N only
  uint32_t status_idx;
  uint32_t acc_off;    // the query's counters: acc + acc_off
  uint32_t pad;
};

// Head launches: `ctr` is one device word that must be zero when the launch
// starts (the dynamic chunk counter); the launch leaves it nonzero.
hipError_t launch_head_args(int Lk, const HeadSegTable &tab, uint64_t nchunks, int grid,
                            unsigned long long *acc, unsigned long long *ctr, hipStream_t st);
hipError_t launch_head_ptr(int Lk, const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                           unsigned long long *acc, unsigned long long *ctr, hipStream_t st);
hipError_t launch_finalize(int Lk, const FinQuery &single, const FinQuery *qs, int nq,
                           const unsigned long long *acc, uint64_t *out, pi_status *status,
                           hipStream_t st);
hipError_t launch_zero(unsigned long long *p, uint64_t n, hipStream_t st);
// Queries of 1 to 6 limbs together: one head launch whose chunks run at their
// own query's limb count (segments in device memory), and one finalize launch
// of a workgroup per query.
constexpr int kFusedMaxL = 6;
hipError_t launch_head_fused(const HeadSeg *segs, int nseg, uint64_t nchunks, int grid,
                             unsigned long long *acc, unsigned long long *ctr, hipStream_t st);
hipError_t launch_finalize_fused(const FinQuery *qs, int nq, const unsigned long long *acc,
                                 uint64_t *out, pi_status *status, hipStream_t st);
int head_occupancy_fused();
// Workgroups of the head kernel instance for Lk limbs that fit on one CU
// (by_value: the instance taking its segment table as a kernel argument).
int head_occupancy(int Lk, bool by_value);
// The device address of the static scratch array on the current device (looked
// up once per device) and its size in 64-bit words.
hipError_t static_scratch(unsigned long long **ptr, uint32_t *words);
hipError_t launch_combine(const uint64_t *parts, int count, int Lq, uint32_t P, uint32_t w,
                          uint64_t nterms, uint32_t J, uint64_t *out, pi_status *status,
                          hipStream_t st);

}  // namespace pibbp
