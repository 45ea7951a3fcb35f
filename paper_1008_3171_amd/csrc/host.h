// Host-side planning shared by the C ABI entry points and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pibbp.h"
#include "plan.h"

namespace pibbp {
namespace host {

// One extraction (or slice) planned on the host: the head and tail index
// ranges of every series, N's head part, and the limb counts.
struct QueryPlan {
  int formula;
  uint64_t d;
  uint32_t P, w, Lq;
  int Lk;                   // limb count of the kernel instance used
  uint64_t hk0[7], hk1[7];  // head ranges
  uint64_t tk0[7], tk1[7];  // tail ranges
  uint64_t nhead;
};

int make_plan(int formula, uint64_t n, uint32_t w, uint32_t P, uint32_t jmask, uint64_t k0,
              uint64_t k1, QueryPlan *qp);
// The head segments of a plan into out[0 .. kMaxArgSegs), returning their count;
// or appended to a vector.
int head_segments(const QueryPlan &qp, uint32_t acc_off, HeadSeg *out);
void head_segments(const QueryPlan &qp, uint32_t acc_off, std::vector<HeadSeg> &out);
uint64_t number_chunks(HeadSeg *segs, size_t nseg, uint32_t run_cap, uint64_t chunk_base);
uint64_t number_chunks(std::vector<HeadSeg> &segs, uint32_t run_cap, uint64_t chunk_base);
uint32_t pick_run(uint64_t head_terms, int grid, uint32_t cap);
uint32_t run_cap_for(int Lk);
uint32_t run_cap_fused();
uint32_t min_run_cap(uint64_t head_terms);
FinQuery fin_query(const QueryPlan &qp, uint64_t out_off, uint32_t status_mode, uint32_t sidx,
                   uint32_t acc_off);
int resident_grid(int Lk, bool by_value);
int resident_grid_fused();
int hip_err(hipError_t e);

}  // namespace host
}  // namespace pibbp
