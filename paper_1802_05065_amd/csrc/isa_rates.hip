// isa_rates.hip -- issue-rate microbenchmark of the VALU instructions the
// integrator is built from (gfx950).
//
// Each lane runs 8 independent dependency chains of one instruction, written
// as inline assembly so that the compiler neither folds nor reorders them;
// with 8 waves per SIMD the chains hide latency and the measured rate is the
// instruction's throughput.  Rates are printed absolute (lane-ops/s) and
// relative to v_fma_f32, i.e. each instruction's cost in v_fma_f32 issue
// slots.  "pair" tests issue two different instructions per chain step to
// show whether they overlap (cost of the pair < sum of the two); the
// "cross-wave" line does the same with the two instructions in different
// waves of the SIMD.
//
// usage: isa_rates
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e = (x);                                                   \
    if (e != hipSuccess) {                                                \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));         \
      return 1;                                                           \
    }                                                                     \
  } while (0)

constexpr int kChains = 8;
constexpr int kIters = 1024;
constexpr int kThreads = 256;

// One chain step per op.  Operands: x, y (32-bit chains), d (64-bit chain),
// a, b (64-bit constants) and p, q (32-bit constants).
#define OP_LIST(X)                                                                     \
  X(fma_f32, "v_fma_f32 %[x], %[x], %[p], %[q]", 1)                                   \
  X(add_f32, "v_add_f32 %[x], %[x], %[p]", 1)                                         \
  X(mul_f32, "v_mul_f32 %[x], %[x], %[p]", 1)                                         \
  X(sin_f32, "v_sin_f32 %[x], %[x]", 1)                                               \
  X(cos_f32, "v_cos_f32 %[x], %[x]", 1)                                               \
  X(log_f32, "v_log_f32 %[x], %[x]", 1)                                               \
  X(sqrt_f32, "v_sqrt_f32 %[x], %[x]", 1)                                             \
  X(cvt_f32_u32, "v_cvt_f32_u32 %[x], %[x]", 1)                                       \
  X(xor_b32, "v_xor_b32 %[x], %[x], %[p]", 1)                                         \
  X(bitop3_b32, "v_bitop3_b32 %[x], %[x], %[p], %[q] bitop3:0x96", 1)                 \
  X(add_u32, "v_add_u32 %[x], %[x], %[p]", 1)                                         \
  X(mul_lo_u32, "v_mul_lo_u32 %[x], %[x], %[p]", 1)                                   \
  X(mul_hi_u32, "v_mul_hi_u32 %[x], %[x], %[p]", 1)                                   \
  X(fma_f64, "v_fma_f64 %[d], %[d], %[a], %[b]", 1)                                   \
  X(add_f64, "v_add_f64 %[d], %[d], %[a]", 1)                                         \
  X(mad_u64_u32, "v_mad_u64_u32 %[d], vcc, %[x], %[p], %[d]", 1)                      \
  X(cvt_f32_f64_pair, "v_cvt_f32_f64 %[x], %[d]\n v_cvt_f64_f32 %[d], %[x]", 2)       \
  X(fma_f32_sin, "v_fma_f32 %[x], %[x], %[p], %[q]\n v_sin_f32 %[y], %[y]", 2)        \
  X(fma_f32_mulhi, "v_fma_f32 %[x], %[x], %[p], %[q]\n v_mul_hi_u32 %[y], %[y], %[p]", 2) \
  X(fma_f32_fma_f64, "v_fma_f64 %[d], %[d], %[a], %[b]\n v_fma_f32 %[x], %[x], %[p], %[q]", 2) \
  X(fma_f32_mad64, "v_mad_u64_u32 %[d], vcc, %[y], %[p], %[d]\n v_fma_f32 %[x], %[x], %[p], %[q]", 2) \
  X(sin_mad64, "v_mad_u64_u32 %[d], vcc, %[y], %[p], %[d]\n v_sin_f32 %[x], %[x]", 2)      \
  X(fma_f32_s, "v_fma_f32 %[x], %[x], %[ps], %[q]", 1)                                \
  X(fma_f32_ss, "v_fma_f32 %[x], %[x], %[ps], %[ps]", 1)                              \
  X(fmac_f32_s, "v_fmac_f32 %[x], %[ps], %[y]", 1)                                    \
  X(fmac_f32_v, "v_fmac_f32 %[x], %[q], %[y]", 1)                                     \
  X(fmamk_f32, "v_fmamk_f32 %[x], %[x], 0x3f7fbe77, %[q]", 1)                         \
  X(mad_u64_u32_s0, "v_mad_u64_u32 %[d], vcc, %[x], %[ps], 0", 1)                     \
  X(bitop3_b32_s, "v_bitop3_b32 %[x], %[x], %[y], %[ps] bitop3:0x96", 1)               \
  X(sub_f32, "v_sub_f32 %[x], %[x], %[y]", 1)                                         \
  X(sqrt_f32_neg, "v_sqrt_f32_e64 %[x], -%[x]", 1)                                     \
  X(log_f32_e64, "v_log_f32_e64 %[x], |%[x]|", 1)                                      \
  X(alignbit_b32, "v_alignbit_b32 %[x], %[ps], %[x], 9", 1)                            \
  X(max3_f32, "v_max3_f32 %[x], %[x], %[y], %[p]", 1)                                  \
  X(max_f32, "v_max_f32 %[x], %[x], %[y]", 1)                                         \
  X(cvt_f32_f64, "v_cvt_f32_f64 %[x], %[d]", 1)                                       \
  X(sin_fmac_pair, "v_sin_f32 %[x], %[x]\n v_fmac_f32 %[y], %[ps], %[y]", 2)            \
  X(sin_add_pair, "v_sin_f32 %[x], %[x]\n v_add_f32 %[y], %[y], %[p]", 2)

#define DECL(name, text, n)                                                           \
  __global__ __launch_bounds__(kThreads) void k_##name(float* out, float seed) {     \
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;                           \
    float x[kChains], y[kChains];                                                     \
    double d[kChains];                                                                \
    const double a = 0.999 + 1e-9 * seed, b = 1e-3 * seed;                            \
    const float p = 0.999f + 1e-9f * seed, q = 1e-3f * seed;                          \
    for (int c = 0; c < kChains; ++c) {                                               \
      x[c] = 0.25f + 1e-7f * (float)(t + c);                                          \
      y[c] = 0.5f + 1e-7f * (float)(t + c);                                           \
      d[c] = 0.25 + 1e-7 * (double)(t + c);                                           \
    }                                                                                 \
    for (int i = 0; i < kIters; ++i) {                                                \
      _Pragma("unroll") for (int c = 0; c < kChains; ++c)                             \
        asm volatile(text : [x] "+v"(x[c]), [y] "+v"(y[c]), [d] "+v"(d[c])            \
                     : [a] "v"(a), [b] "v"(b), [p] "v"(p), [q] "v"(q), [ps] "s"(p)     \
                     : "vcc");                                                        \
    }                                                                                 \
    float acc = 0.f;                                                                  \
    for (int c = 0; c < kChains; ++c) acc += x[c] + y[c] + (float)d[c];               \
    out[t] = acc;                                                                     \
  }

OP_LIST(DECL)

struct Entry {
  const char* name;
  void (*kernel)(float*, float);
  int insts;
  double rate;  // chain steps per second (all lanes)
};

#define ENTRY(name, text, n) {#name, k_##name, n, 0.0},
static Entry g_entries[] = {OP_LIST(ENTRY)};

// Cross-wave overlap: the even waves of each workgroup run v_sin_f32 chains
// and the odd ones v_fmac_f32 chains, as many steps each.  If the SIMD
// issued a transcendental of one wave beside a VALU instruction of another,
// the launch would take as long as its slower half; if they share the issue
// slots, as long as the two halves one after the other.
__global__ __launch_bounds__(kThreads) void k_split_sin_fmac(float* out, float seed) {
  const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
  float x[kChains];
  const float p = 0.999f + 1e-9f * seed;
  for (int c = 0; c < kChains; ++c) x[c] = 0.25f + 1e-7f * (float)(t + c);
  if (((threadIdx.x / 64) & 1) == 0) {
    for (int i = 0; i < kIters; ++i) {
      _Pragma("unroll") for (int c = 0; c < kChains; ++c)
        asm volatile("v_sin_f32 %[x], %[x]" : [x] "+v"(x[c]));
    }
  } else {
    for (int i = 0; i < kIters; ++i) {
      _Pragma("unroll") for (int c = 0; c < kChains; ++c)
        asm volatile("v_fmac_f32 %[x], %[ps], %[x]" : [x] "+v"(x[c]) : [ps] "s"(p));
    }
  }
  float acc = 0.f;
  for (int c = 0; c < kChains; ++c) acc += x[c];
  out[t] = acc;
}

static int measure(Entry& e, float* out, int groups, hipEvent_t e0, hipEvent_t e1) {
  hipLaunchKernelGGL(e.kernel, dim3(groups), dim3(kThreads), 0, 0, out, 1.0f);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e0, 0));
  for (int rep = 0; rep < 4; ++rep)
    hipLaunchKernelGGL(e.kernel, dim3(groups), dim3(kThreads), 0, 0, out, 1.0f);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  e.rate = 4.0 * groups * kThreads * (double)kIters * kChains / (ms * 1e-3);
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
  const int n = (int)(sizeof(g_entries) / sizeof(g_entries[0]));
  for (int i = 0; i < n; ++i)
    if (measure(g_entries[i], out, groups, e0, e1)) return 1;
  Entry split{"split_sin_fmac", k_split_sin_fmac, 1, 0.0};
  if (measure(split, out, groups, e0, e1)) return 1;
  Entry sin_only{}, fmac_only{};
  for (int i = 0; i < n; ++i) {
    if (std::strcmp(g_entries[i].name, "sin_f32") == 0) sin_only = g_entries[i];
    if (std::strcmp(g_entries[i].name, "fmac_f32_s") == 0) fmac_only = g_entries[i];
  }
  const double fma_rate = g_entries[0].rate;
  std::printf("gfx950 VALU issue rates: %d CUs, 8 waves/SIMD, %d chains x %d steps per lane\n",
              cus, kChains, kIters);
  std::printf("%-20s %6s %16s %22s\n", "chain step", "insts", "T steps/s",
              "v_fma_f32 slots/step");
  for (int i = 0; i < n; ++i)
    std::printf("%-20s %6d %16.2f %22.2f\n", g_entries[i].name, g_entries[i].insts,
                g_entries[i].rate * 1e-12, fma_rate / g_entries[i].rate);
  std::printf("v_fma_f32: %.2f T lane-op/s = %.1f lane-ops per CU per ns\n", fma_rate * 1e-12,
              fma_rate / cus * 1e-9);
  // times per lane-instruction, relative to the split launch's
  const double t_split = 1.0 / split.rate;
  const double t_serial = 0.5 / sin_only.rate + 0.5 / fmac_only.rate;
  const double t_overlap = std::max(0.5 / sin_only.rate, 0.5 / fmac_only.rate);
  std::printf("cross-wave: even waves v_sin_f32, odd waves v_fmac_f32 (s): %.2f T lane-op/s; "
              "time %.3f of the halves one after the other, %.3f of the slower half alone\n",
              split.rate * 1e-12, t_split / t_serial, t_split / t_overlap);
  CHECK(hipFree(out));
  return 0;
}
