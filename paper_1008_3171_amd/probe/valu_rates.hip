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

#define KERNELF64(NAME, ASM)                                                     \
  __global__ void NAME(uint32_t *out, uint32_t seed) {                           \
    const double b = 1.0 + (double)((seed + blockIdx.x) & 7u) * 0x1p-40;         \
    double a[kChains];                                                           \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = 1.5 + threadIdx.x + c; \
    for (int i = 0; i < kIter; ++i) {                                            \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b)); \
    }                                                                            \
    double s = 0;                                                                \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s += a[c];               \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(int64_t)s;           \
  }

// One exact modular squaring with doubling in binary64, y = 2^b x^2 - q M,
// as the head kernel's floating-point ladder takes it: the product split
// into H + Lo with an FMA, q = rint(H / M) from a reciprocal, the remainder
// from a second FMA. KCH independent chains per lane; each step is seven
// instructions (ldexp, mul, fma, mul, rndne, fma, add).
template <int KCH>
__global__ void k_sqr_f64(uint32_t *out, uint32_t seed) {
  const double M = (double)((1ull << 39) + 2u * (seed + blockIdx.x) + 1u);
  const double inv = 1.0 / M;
  double x[KCH];
#pragma unroll
  for (int c = 0; c < KCH; ++c) x[c] = (double)(threadIdx.x * 977u + c * 131u + seed);
  for (int i = 0; i < kIter; ++i) {
#pragma unroll
    for (int c = 0; c < KCH; ++c) {
      const double xs = __builtin_amdgcn_ldexp(x[c], (int)((i >> c) & 1));
      const double h = __dmul_rn(x[c], xs);
      const double lo = __builtin_fma(x[c], xs, -h);
      const double q = __builtin_rint(__dmul_rn(h, inv));
      x[c] = __dadd_rn(__builtin_fma(-q, M, h), lo);
    }
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < KCH; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(int64_t)s;
}

KERNEL64(k_mad_u64_u32, "v_mad_u64_u32 %0, vcc, %1, %1, %0")
KERNEL32(k_mul_lo_u32, "v_mul_lo_u32 %0, %0, %1")
KERNEL32(k_mul_hi_u32, "v_mul_hi_u32 %0, %0, %1")
KERNEL32(k_add_u32, "v_add_u32 %0, %0, %1")
KERNEL32(k_alignbit_b32, "v_alignbit_b32 %0, %0, %1, 27")
KERNEL32(k_bfe_u32, "v_bfe_u32 %0, %0, %1, 1")
KERNEL64(k_lshrrev_b64, "v_lshrrev_b64 %0, %1, %0")
KERNEL64(k_lshl_add_u64, "v_lshl_add_u64 %0, %0, 1, %0")
KERNELF64(k_fma_f64, "v_fma_f64 %0, %0, %1, %0")
KERNELF64(k_mul_f64, "v_mul_f64 %0, %0, %1")
KERNELF64(k_add_f64, "v_add_f64 %0, %0, %1")
KERNELF64(k_rndne_f64, "v_rndne_f64 %0, %0")
KERNELF64(k_floor_f64, "v_floor_f64 %0, %0")
KERNELF64(k_ldexp_f64, "v_ldexp_f64 %0, %0, 0")

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
            {"v_lshrrev_b64", k_lshrrev_b64}, {"v_lshl_add_u64", k_lshl_add_u64},
            {"v_fma_f64", k_fma_f64},         {"v_mul_f64", k_mul_f64},
            {"v_add_f64", k_add_f64},         {"v_rndne_f64", k_rndne_f64},
            {"v_floor_f64", k_floor_f64},     {"v_ldexp_f64", k_ldexp_f64}};
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
  // The binary64 squaring step: 7 instructions per step and chain.
  struct {
    const char *name;
    kfn f;
    int chains;
  } st[] = {{"sqr_f64_chains1", k_sqr_f64<1>, 1}, {"sqr_f64_chains2", k_sqr_f64<2>, 2},
            {"sqr_f64_chains4", k_sqr_f64<4>, 4}};
  for (auto &k : st) {
    hipLaunchKernelGGL(k.f, dim3(blocks), dim3(threads), 0, 0, d, 12345u);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int r = 0; r < 3; ++r) hipLaunchKernelGGL(k.f, dim3(blocks), dim3(threads), 0, 0, d, 777u + r);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms = 0;
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double steps = 3.0 * blocks * threads * (double)kIter * k.chains;
    printf("{\"op\": \"%s\", \"steps_per_s\": %.4e, \"instr_per_step\": 7, "
           "\"frac_of_full_rate\": %.3f}\n",
           k.name, steps / (ms * 1e-3), 7.0 * steps / (ms * 1e-3) / peak);
  }
  CK(hipFree(d));
  return 0;
}
