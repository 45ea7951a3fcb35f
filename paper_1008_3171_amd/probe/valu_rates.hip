// Issue rate of VALU instructions on the device this runs on, the denominator
// of the head kernel's roofline.
//
// For each opcode (or mix of opcodes) every lane runs 8 independent chains
// (compute-only inline asm, no memory operands, so nothing is removed or
// merged), 256 threads per workgroup and 32 workgroups per CU. The launch is
// timed with HIP events; inside it, the first wave of block 0 reads the
// shader-clock counter (s_memtime) and the constant-rate counter
// (s_memrealtime) at its start and end, which gives the shader clock the
// kernel actually ran at. Reported per line (one JSON object each):
//   lane_ops_per_s        instructions x 64 lanes per second, chip-wide;
//   per_clk_per_cu        the same per shader clock per CU (64 = one wave64
//                         instruction per SIMD every 4 clocks on 4 SIMDs);
//   clock_ghz             the measured shader clock;
//   frac_of_full_rate     lane_ops_per_s / (CUs x 64 x the attribute clock).
// Mixed lines interleave chains of two opcodes; if the two can issue in the
// same cycle, per_clk_per_cu of the mix exceeds that of either alone.
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
constexpr int kThreads = 256;

// out layout: [0, blocks*threads) per-thread results; then 4 words of clock
// samples (memtime start, memtime end, realtime start, realtime end) as
// uint64 pairs.
struct Clock {
  uint64_t t0, r0;
};
__device__ __forceinline__ Clock clock_start() {
  Clock c;
  c.t0 = __builtin_amdgcn_s_memtime();
  c.r0 = __builtin_amdgcn_s_memrealtime();
  return c;
}
__device__ __forceinline__ void clock_end(const Clock &c, uint64_t *clk) {
  const uint64_t t1 = __builtin_amdgcn_s_memtime();
  const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk[0] = t1 - c.t0;
    clk[1] = r1 - c.r0;
  }
}

#define KERNEL32(NAME, ASM)                                                       \
  __global__ void NAME(uint32_t *out, uint64_t *clk, uint32_t seed) {             \
    const Clock c0 = clock_start();                                               \
    uint32_t b = (seed * 3u + blockIdx.x) | 1u;                                   \
    uint32_t a[kChains];                                                          \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = seed + threadIdx.x * 7u + c; \
    for (int i = 0; i < kIter; ++i) {                                             \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b) : "vcc"); \
    }                                                                             \
    uint32_t s = 0;                                                               \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s ^= a[c];                \
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;                               \
    clock_end(c0, clk);                                                           \
  }
#define KERNEL64(NAME, ASM)                                                       \
  __global__ void NAME(uint32_t *out, uint64_t *clk, uint32_t seed) {             \
    const Clock c0 = clock_start();                                               \
    uint32_t b = (seed * 3u + blockIdx.x) | 1u;                                   \
    uint64_t a[kChains];                                                          \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = seed + threadIdx.x * 7u + c; \
    for (int i = 0; i < kIter; ++i) {                                             \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b) : "vcc"); \
    }                                                                             \
    uint64_t s = 0;                                                               \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s ^= a[c];                \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(s ^ (s >> 32));       \
    clock_end(c0, clk);                                                           \
  }
#define KERNELF64(NAME, ASM)                                                      \
  __global__ void NAME(uint32_t *out, uint64_t *clk, uint32_t seed) {             \
    const Clock c0 = clock_start();                                               \
    const double b = 1.0 + (double)((seed + blockIdx.x) & 7u) * 0x1p-40;          \
    double a[kChains];                                                            \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = 1.5 + threadIdx.x + c; \
    for (int i = 0; i < kIter; ++i) {                                             \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b)); \
    }                                                                             \
    double s = 0;                                                                 \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s += a[c];                \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(int64_t)s;            \
    clock_end(c0, clk);                                                           \
  }
#define KERNELF32(NAME, ASM)                                                      \
  __global__ void NAME(uint32_t *out, uint64_t *clk, uint32_t seed) {             \
    const Clock c0 = clock_start();                                               \
    const float b = 1.0f + (float)((seed + blockIdx.x) & 7u) * 0x1p-20f;          \
    float a[kChains];                                                             \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = 1.5f + threadIdx.x + c; \
    for (int i = 0; i < kIter; ++i) {                                             \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c) asm volatile(ASM : "+v"(a[c]) : "v"(b)); \
    }                                                                             \
    float s = 0;                                                                  \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) s += a[c];                \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(int32_t)s;            \
    clock_end(c0, clk);                                                           \
  }
// Two opcodes interleaved: kChains/2 chains of each, alternating in the
// unrolled loop body (one on 64-bit doubles, one on 32-bit words).
#define KERNELMIX_F64_U32(NAME, ASMF, ASMU)                                       \
  __global__ void NAME(uint32_t *out, uint64_t *clk, uint32_t seed) {             \
    const Clock c0 = clock_start();                                               \
    const double bf = 1.0 + (double)((seed + blockIdx.x) & 7u) * 0x1p-40;         \
    const uint32_t bu = (seed * 3u + blockIdx.x) | 1u;                            \
    double af[kChains / 2];                                                       \
    uint32_t au[kChains / 2];                                                     \
    _Pragma("unroll") for (int c = 0; c < kChains / 2; ++c) {                     \
      af[c] = 1.5 + threadIdx.x + c;                                              \
      au[c] = seed + threadIdx.x * 7u + c;                                        \
    }                                                                             \
    for (int i = 0; i < kIter; ++i) {                                             \
      _Pragma("unroll") for (int c = 0; c < kChains / 2; ++c) {                   \
        asm volatile(ASMF : "+v"(af[c]) : "v"(bf));                               \
        asm volatile(ASMU : "+v"(au[c]) : "v"(bu) : "vcc");                       \
      }                                                                           \
    }                                                                             \
    double s = 0;                                                                 \
    uint32_t t = 0;                                                               \
    _Pragma("unroll") for (int c = 0; c < kChains / 2; ++c) {                     \
      s += af[c];                                                                 \
      t ^= au[c];                                                                 \
    }                                                                             \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(int64_t)s ^ t;        \
    clock_end(c0, clk);                                                           \
  }
#define KERNELMIX_U64_U32(NAME, ASM64, ASMU)                                      \
  __global__ void NAME(uint32_t *out, uint64_t *clk, uint32_t seed) {             \
    const Clock c0 = clock_start();                                               \
    const uint32_t bu = (seed * 3u + blockIdx.x) | 1u;                            \
    uint64_t a6[kChains / 2];                                                     \
    uint32_t au[kChains / 2];                                                     \
    _Pragma("unroll") for (int c = 0; c < kChains / 2; ++c) {                     \
      a6[c] = seed + threadIdx.x * 5u + c;                                        \
      au[c] = seed + threadIdx.x * 7u + c;                                        \
    }                                                                             \
    for (int i = 0; i < kIter; ++i) {                                             \
      _Pragma("unroll") for (int c = 0; c < kChains / 2; ++c) {                   \
        asm volatile(ASM64 : "+v"(a6[c]) : "v"(bu) : "vcc");                      \
        asm volatile(ASMU : "+v"(au[c]) : "v"(bu) : "vcc");                       \
      }                                                                           \
    }                                                                             \
    uint64_t s = 0;                                                               \
    uint32_t t = 0;                                                               \
    _Pragma("unroll") for (int c = 0; c < kChains / 2; ++c) {                     \
      s ^= a6[c];                                                                 \
      t ^= au[c];                                                                 \
    }                                                                             \
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(s ^ (s >> 32)) ^ t;    \
    clock_end(c0, clk);                                                           \
  }

// One exact modular squaring in binary64, y = 2^b x^2 - q M (the head
// kernel's floating-point ladder step, plus its window shift): the product
// split into H + Lo with an FMA, q = rint(H / M) from a reciprocal, the
// remainder from a second FMA. KCH independent chains per lane; each step is
// seven instructions (ldexp, mul, fma, mul, rndne, fma, add).
template <int KCH>
__global__ void k_sqr_f64(uint32_t *out, uint64_t *clk, uint32_t seed) {
  const Clock c0 = clock_start();
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
  clock_end(c0, clk);
}

KERNEL64(k_mad_u64_u32, "v_mad_u64_u32 %0, vcc, %1, %1, %0")
KERNEL32(k_mul_lo_u32, "v_mul_lo_u32 %0, %0, %1")
KERNEL32(k_mul_hi_u32, "v_mul_hi_u32 %0, %0, %1")
KERNEL32(k_mul_u32_u24, "v_mul_u32_u24 %0, %0, %1")
KERNEL32(k_add_u32, "v_add_u32 %0, %0, %1")
KERNEL32(k_sub_u32, "v_sub_u32 %0, %0, %1")
KERNEL32(k_add_co_u32, "v_add_co_u32 %0, vcc, %0, %1")
KERNEL32(k_add3_u32, "v_add3_u32 %0, %0, %1, %0")
KERNEL32(k_xor_b32, "v_xor_b32 %0, %0, %1")
KERNEL32(k_and_b32, "v_and_b32 %0, %0, %1")
KERNEL32(k_lshlrev_b32, "v_lshlrev_b32 %0, 1, %0")
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
KERNELF32(k_fma_f32, "v_fma_f32 %0, %0, %1, %0")
KERNELF32(k_add_f32, "v_add_f32 %0, %0, %1")
KERNELF32(k_mul_f32, "v_mul_f32 %0, %0, %1")
KERNELMIX_F64_U32(k_mix_fma_f64_add_u32, "v_fma_f64 %0, %0, %1, %0", "v_add_u32 %0, %0, %1")
KERNELMIX_F64_U32(k_mix_fma_f64_xor_b32, "v_fma_f64 %0, %0, %1, %0", "v_xor_b32 %0, %0, %1")
KERNELMIX_F64_U32(k_mix_fma_f64_mul_lo_u32, "v_fma_f64 %0, %0, %1, %0", "v_mul_lo_u32 %0, %0, %1")
KERNELMIX_U64_U32(k_mix_mad_u64_add_u32, "v_mad_u64_u32 %0, vcc, %1, %1, %0",
                  "v_add_u32 %0, %0, %1")

typedef void (*kfn)(uint32_t *, uint64_t *, uint32_t);

struct Probe {
  const char *name;
  kfn f;
  double instr;  // instructions per chain step
  int chains;    // chains per lane
};

int main() {
  int dev = 0, cus = 0, clock_khz = 0, wall_khz = 0;
  CK(hipGetDevice(&dev));
  CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  CK(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, dev));
  CK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
  const double peak = (double)cus * 64.0 * clock_khz * 1e3;
  const int blocks = cus * 32;
  uint32_t *d = nullptr;
  uint64_t *clk = nullptr;
  CK(hipMalloc(&d, sizeof(uint32_t) * (size_t)kThreads * blocks));
  CK(hipMalloc(&clk, 2 * sizeof(uint64_t)));
  printf("{\"device\": {\"cus\": %d, \"clock_attr_ghz\": %.3f, \"wall_clock_mhz\": %.1f, "
         "\"full_rate\": %.4e}}\n",
         cus, clock_khz * 1e-6, wall_khz * 1e-3, peak);
  const Probe ps[] = {
      {"v_mad_u64_u32", k_mad_u64_u32, 1, kChains},
      {"v_mul_lo_u32", k_mul_lo_u32, 1, kChains},
      {"v_mul_hi_u32", k_mul_hi_u32, 1, kChains},
      {"v_mul_u32_u24", k_mul_u32_u24, 1, kChains},
      {"v_add_u32", k_add_u32, 1, kChains},
      {"v_sub_u32", k_sub_u32, 1, kChains},
      {"v_add_co_u32", k_add_co_u32, 1, kChains},
      {"v_add3_u32", k_add3_u32, 1, kChains},
      {"v_xor_b32", k_xor_b32, 1, kChains},
      {"v_and_b32", k_and_b32, 1, kChains},
      {"v_lshlrev_b32", k_lshlrev_b32, 1, kChains},
      {"v_alignbit_b32", k_alignbit_b32, 1, kChains},
      {"v_bfe_u32", k_bfe_u32, 1, kChains},
      {"v_lshrrev_b64", k_lshrrev_b64, 1, kChains},
      {"v_lshl_add_u64", k_lshl_add_u64, 1, kChains},
      {"v_fma_f64", k_fma_f64, 1, kChains},
      {"v_mul_f64", k_mul_f64, 1, kChains},
      {"v_add_f64", k_add_f64, 1, kChains},
      {"v_rndne_f64", k_rndne_f64, 1, kChains},
      {"v_floor_f64", k_floor_f64, 1, kChains},
      {"v_ldexp_f64", k_ldexp_f64, 1, kChains},
      {"v_fma_f32", k_fma_f32, 1, kChains},
      {"v_add_f32", k_add_f32, 1, kChains},
      {"v_mul_f32", k_mul_f32, 1, kChains},
      {"mix v_fma_f64 + v_add_u32", k_mix_fma_f64_add_u32, 1, kChains},
      {"mix v_fma_f64 + v_xor_b32", k_mix_fma_f64_xor_b32, 1, kChains},
      {"mix v_fma_f64 + v_mul_lo_u32", k_mix_fma_f64_mul_lo_u32, 1, kChains},
      {"mix v_mad_u64_u32 + v_add_u32", k_mix_mad_u64_add_u32, 1, kChains},
      // the binary64 squaring step: 7 instructions per step and chain
      {"sqr_f64 step, 1 chain", k_sqr_f64<1>, 7, 1},
      {"sqr_f64 step, 2 chains", k_sqr_f64<2>, 7, 2},
      {"sqr_f64 step, 4 chains", k_sqr_f64<4>, 7, 4},
  };
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (const Probe &p : ps) {
    hipLaunchKernelGGL(p.f, dim3(blocks), dim3(kThreads), 0, 0, d, clk, 12345u);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int r = 0; r < 3; ++r)
      hipLaunchKernelGGL(p.f, dim3(blocks), dim3(kThreads), 0, 0, d, clk, 777u + r);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms = 0;
    CK(hipEventElapsedTime(&ms, e0, e1));
    uint64_t c[2];
    CK(hipMemcpy(c, clk, sizeof c, hipMemcpyDeviceToHost));
    const double clock_hz = c[1] ? (double)c[0] / ((double)c[1] / (wall_khz * 1e3)) : 0.0;
    const double ops = 3.0 * blocks * kThreads * (double)kIter * p.chains * p.instr;
    const double rate = ops / (ms * 1e-3);
    printf("{\"op\": \"%s\", \"lane_ops_per_s\": %.4e, \"per_clk_per_cu\": %.2f, "
           "\"clock_ghz\": %.3f, \"frac_of_full_rate\": %.3f}\n",
           p.name, rate, clock_hz > 0 ? rate / clock_hz / cus : 0.0, clock_hz * 1e-9,
           rate / peak);
  }
  CK(hipFree(d));
  CK(hipFree(clk));
  return 0;
}
