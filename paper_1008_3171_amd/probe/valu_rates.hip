// Issue rate of the VALU instructions the head kernel is built from, on the
// device this runs on: for each opcode, every lane runs 8 independent chains
// of it (forced with compute-only inline asm, no memory operands), and the
// rate is reported in lane-operations per second and as a fraction of
// CUs x 64 lanes x peak engine clock.
//
// Output: one JSON object per line.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                   \
  do {                                                                          \
    hipError_t e = (x);                                                         \
    if (e != hipSuccess) {                                                      \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e), __LINE__); \
      exit(1);                                                                  \
    }                                                                           \
  } while (0)

constexpr int kIter = 2048;
constexpr int kChains = 8;

#define KERNEL32(NAME, ASM)                                                      \
  __global__ void NAME(uint32_t *out, uint32_t seed) {                           \
    uint32_t b = (seed * 3u + blockIdx.x) | 1u;                                  \
    uint32_t a[kChains];                                                         \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = seed + threadIdx.x * 7u + c; \
    for (int i = 0; i < kIter; ++i) {                                            \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b)); \
    }                                                                            \
    uint32_t s = 0;                                                              \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s ^= a[c];               \
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;                              \
  }
#define KERNEL64(NAME, ASM)                                                      \
  __global__ void NAME(uint32_t *out, uint32_t seed) {                           \
    uint32_t b = (seed * 3u + blockIdx.x) | 1u;                                  \
    uint64_t a[kChains];                                                         \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = seed + threadIdx.x * 7u + c; \
    for (int i = 0; i < kIter; ++i) {                                            \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b) : "vcc"); \
    }                                                                            \
    uint64_t s = 0;                                                              \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s ^= a[c];               \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(s ^ (s >> 32));      \
  }

KERNEL64(k_mad_u64_u32, "v_mad_u64_u32 %0, vcc, %1, %1, %0")
KERNEL32(k_mul_lo_u32, "v_mul_lo_u32 %0, %0, %1")
KERNEL32(k_mul_hi_u32, "v_mul_hi_u32 %0, %0, %1")
KERNEL32(k_add_u32, "v_add_u32 %0, %0, %1")
KERNEL32(k_alignbit_b32, "v_alignbit_b32 %0, %0, %1, 27")
KERNEL32(k_bfe_u32, "v_bfe_u32 %0, %0, %1, 1")
KERNEL64(k_lshrrev_b64, "v_lshrrev_b64 %0, %1, %0")
KERNEL64(k_lshl_add_u64, "v_lshl_add_u64 %0, %0, 1, %0")

typedef void (*kfn)(uint32_t *, uint32_t);

int main() {
  int dev = 0, cus = 0, clock_khz = 0;
  CK(hipGetDevice(&dev));
  CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  CK(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, dev));
  const double peak = (double)cus * 64.0 * clock_khz * 1e3;
  const int threads = 256, blocks = cus * 32;
  uint32_t *d = nullptr;
  CK(hipMalloc(&d, sizeof(uint32_t) * (size_t)threads * blocks));
  struct {
    const char *name;
    kfn f;
  } ks[] = {{"v_mad_u64_u32", k_mad_u64_u32}, {"v_mul_lo_u32", k_mul_lo_u32},
            {"v_mul_hi_u32", k_mul_hi_u32},   {"v_add_u32", k_add_u32},
            {"v_alignbit_b32", k_alignbit_b32}, {"v_bfe_u32", k_bfe_u32},
            {"v_lshrrev_b64", k_lshrrev_b64}, {"v_lshl_add_u64", k_lshl_add_u64}};
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (auto &k : ks) {
    hipLaunchKernelGGL(k.f, dim3(blocks), dim3(threads), 0, 0, d, 12345u);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int r = 0; r < 3; ++r) hipLaunchKernelGGL(k.f, dim3(blocks), dim3(threads), 0, 0, d, 777u + r);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms = 0;
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double ops = 3.0 * blocks * threads * (double)kIter * kChains;
    printf("{\"op\": \"%s\", \"lane_ops_per_s\": %.4e, \"frac_of_full_rate\": %.3f, "
           "\"full_rate\": %.4e}\n",
           k.name, ops / (ms * 1e-3), ops / (ms * 1e-3) / peak, peak);
  }
  CK(hipFree(d));
  return 0;
}
