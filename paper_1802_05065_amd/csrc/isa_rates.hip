// isa_rates.hip -- issue-rate microbenchmark of the VALU instructions the
// integrator is made of (gfx950).  Each thread runs 8 independent dependency
// chains of one operation; with 8 waves per SIMD the chains hide latency, so
// the measured rate is the throughput.  Rates are reported relative to a
// chain of v_fma_f32, the full-rate reference, which gives each instruction's
// cost in full-rate issue slots.  A "pair" test interleaves v_fma_f32 with a
// transcendental to show whether the two share issue slots.
//
// usage: isa_rates  (prints one line per operation)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e = (x);                                                   \
    if (e != hipSuccess) {                                                \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));         \
      return 1;                                                           \
    }                                                                     \
  } while (0)

constexpr int kChains = 8;
constexpr int kIters = 2048;
constexpr int kThreads = 256;

enum Op {
  OP_FMA_F32, OP_SIN_F32, OP_LOG_F32, OP_SQRT_F32, OP_MAD_U64_U32, OP_MUL_HI_U32,
  OP_XOR, OP_FMA_F64, OP_CVT_F32_F64, OP_CVT_F32_U32, OP_PAIR_FMA_SIN, OP_PAIR_FMA_MAD64,
  OP_COUNT
};

static const char* kNames[OP_COUNT] = {
    "v_fma_f32", "v_sin_f32", "v_log_f32", "v_sqrt_f32", "v_mad_u64_u32 (+xor)",
    "v_mul_hi_u32 (+add)", "v_xor_b32", "v_fma_f64", "v_cvt_f32_f64 (+fma_f64)",
    "v_cvt_f32_u32 (+add)",
    "v_fma_f32 + v_sin_f32 (pair)", "v_fma_f32 + v_mad_u64_u32 (pair)"};
// VALU instructions per chain step (the v_mad_u64_u32 step also xors the two
// halves; the conversions come with one add)
static const int kInstPerStep[OP_COUNT] = {1, 1, 1, 1, 2, 2, 1, 1, 2, 2, 2, 3};

template <int OP>
__global__ __launch_bounds__(kThreads) void rate_kernel(float* out, float seed) {
  const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
  float f[kChains], g[kChains];
  double d[kChains];
  uint32_t u[kChains];
  for (int c = 0; c < kChains; ++c) {
    f[c] = seed * (float)(t + c + 1) * 1e-9f;
    g[c] = f[c] + 0.25f;
    d[c] = (double)f[c];
    u[c] = t * 2654435761u + (uint32_t)c;
  }
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == OP_FMA_F32) {
        f[c] = __builtin_fmaf(f[c], 0.999f, 1e-3f);
      } else if constexpr (OP == OP_SIN_F32) {
        f[c] = __builtin_amdgcn_sinf(f[c]);
      } else if constexpr (OP == OP_LOG_F32) {
        f[c] = __builtin_amdgcn_logf(f[c]);
      } else if constexpr (OP == OP_SQRT_F32) {
        f[c] = __builtin_amdgcn_sqrtf(f[c]);
      } else if constexpr (OP == OP_MAD_U64_U32) {
        const uint64_t p = (uint64_t)u[c] * 0xD2511F53u;
        u[c] = (uint32_t)p ^ (uint32_t)(p >> 32);
      } else if constexpr (OP == OP_MUL_HI_U32) {
        u[c] = __umulhi(u[c], 0xCD9E8D57u) + 1u;
      } else if constexpr (OP == OP_XOR) {
        u[c] ^= (uint32_t)i * 0x9E3779B9u;
      } else if constexpr (OP == OP_FMA_F64) {
        d[c] = __builtin_fma(d[c], 0.999, 1e-3);
      } else if constexpr (OP == OP_CVT_F32_F64) {
        f[c] = (float)d[c];
        d[c] = __builtin_fma(d[c], 0.999, 1e-3);
      } else if constexpr (OP == OP_CVT_F32_U32) {
        f[c] = (float)(u[c] + (uint32_t)__float_as_uint(f[c]));
      } else if constexpr (OP == OP_PAIR_FMA_SIN) {
        f[c] = __builtin_fmaf(f[c], 0.999f, 1e-3f);
        g[c] = __builtin_amdgcn_sinf(g[c]);
      } else if constexpr (OP == OP_PAIR_FMA_MAD64) {
        f[c] = __builtin_fmaf(f[c], 0.999f, 1e-3f);
        const uint64_t p = (uint64_t)u[c] * 0xD2511F53u;
        u[c] = (uint32_t)p ^ (uint32_t)(p >> 32);
      }
    }
  }
  float acc = 0.f;
  for (int c = 0; c < kChains; ++c) acc += f[c] + g[c] + (float)d[c] + (float)u[c];
  out[t] = acc;
}

template <int OP>
static int run(float* out, int groups, hipEvent_t e0, hipEvent_t e1, double* ops_per_s) {
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(groups), dim3(kThreads), 0, 0, out, 1.0f);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e0, 0));
  for (int rep = 0; rep < 5; ++rep)
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(groups), dim3(kThreads), 0, 0, out, 1.0f);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const double lane_steps = 5.0 * groups * kThreads * (double)kIters * kChains;
  *ops_per_s = lane_steps / (ms * 1e-3);
  return 0;
}

int main() {
  int dev = 0, cus = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int groups = cus * 4 * 8 * 64 / kThreads;  // 8 waves per SIMD
  float* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(float) * groups * kThreads));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  double r[OP_COUNT];
  if (run<OP_FMA_F32>(out, groups, e0, e1, &r[OP_FMA_F32]) ||
      run<OP_SIN_F32>(out, groups, e0, e1, &r[OP_SIN_F32]) ||
      run<OP_LOG_F32>(out, groups, e0, e1, &r[OP_LOG_F32]) ||
      run<OP_SQRT_F32>(out, groups, e0, e1, &r[OP_SQRT_F32]) ||
      run<OP_MAD_U64_U32>(out, groups, e0, e1, &r[OP_MAD_U64_U32]) ||
      run<OP_MUL_HI_U32>(out, groups, e0, e1, &r[OP_MUL_HI_U32]) ||
      run<OP_XOR>(out, groups, e0, e1, &r[OP_XOR]) ||
      run<OP_FMA_F64>(out, groups, e0, e1, &r[OP_FMA_F64]) ||
      run<OP_CVT_F32_F64>(out, groups, e0, e1, &r[OP_CVT_F32_F64]) ||
      run<OP_CVT_F32_U32>(out, groups, e0, e1, &r[OP_CVT_F32_U32]) ||
      run<OP_PAIR_FMA_SIN>(out, groups, e0, e1, &r[OP_PAIR_FMA_SIN]) ||
      run<OP_PAIR_FMA_MAD64>(out, groups, e0, e1, &r[OP_PAIR_FMA_MAD64]))
    return 1;
  std::printf("CUs %d, 8 waves/SIMD, %d chains x %d iterations per lane\n", cus, kChains,
              kIters);
  std::printf("%-34s %6s %14s %18s\n", "operation", "insts", "Gsteps/s",
              "slots per step");
  for (int op = 0; op < OP_COUNT; ++op)
    std::printf("%-34s %6d %14.1f %18.2f\n", kNames[op], kInstPerStep[op], r[op] * 1e-9,
                r[OP_FMA_F32] / r[op]);
  std::printf("v_fma_f32 rate = %.2f Tlane-op/s (clock-equivalent %.3f GHz at 64 lanes/CU)\n",
              r[OP_FMA_F32] * 1e-12, r[OP_FMA_F32] / (64.0 * cus) * 1e-9);
  CHECK(hipFree(out));
  return 0;
}
