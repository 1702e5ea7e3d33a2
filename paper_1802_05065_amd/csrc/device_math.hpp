// device_math.hpp -- per-replica arithmetic of the integrator on gfx950:
// counter-based generator, Box-Muller normals and the Euler-Maruyama step of
// Algorithms 1 and 3 (arXiv:1802.05065, Sect. III.B), in FP64 and in FP32
// with a compensated phase.
//
// Every file that includes this is compiled with -ffp-contract=off, so the
// FP64 expressions below round exactly as written (no implicit FMA).  The
// FP32C path requests fused operations explicitly where it wants them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace fpt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The 32x32 -> 64
// products map to v_mad_u64_u32; with a wave-uniform key the key schedule
// lives in scalar registers.
struct Words {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1,
                                               uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// Words of block j of replica idx: counter (j lo, j hi, idx lo, idx hi),
// key (seed lo, seed hi).
__device__ __forceinline__ Words replica_words(uint64_t seed, uint64_t idx,
                                               uint64_t j) {
  return philox4x32_10((uint32_t)j, (uint32_t)(j >> 32), (uint32_t)idx,
                       (uint32_t)(idx >> 32), (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// Box-Muller: u = (x + 1/2) 2^-32 in (0, 1); a pair (a, b) of uniforms gives
// sqrt(-2 ln a) (cos 2 pi b, sin 2 pi b).

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void normals_f64(const Words& w, double z[4]) {
  const uint32_t x[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const double a = ((double)x[2 * pair] + 0.5) * 0x1p-32;
    const double b = ((double)x[2 * pair + 1] + 0.5) * 0x1p-32;
    const double radius = sqrt(-2.0 * log(a));
    const double angle = 2.0 * kPi * b;
    double s, c;
    sincos(angle, &s, &c);
    z[2 * pair] = radius * c;
    z[2 * pair + 1] = radius * s;
  }
}

// FP32: hardware transcendentals.  v_log_f32 is log2, v_sin/v_cos_f32 take
// their argument in revolutions, so 2 pi b needs no multiply.
__device__ __forceinline__ void normals_f32(const Words& w, float z[4]) {
  const uint32_t x[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const float a = __builtin_fmaf((float)x[2 * pair], 0x1p-32f, 0x1p-33f);
    const float b = __builtin_fmaf((float)x[2 * pair + 1], 0x1p-32f, 0x1p-33f);
    // -2 ln a = -2 ln(2) log2(a)
    const float radius =
        __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(a));
    z[2 * pair] = radius * __builtin_amdgcn_cosf(b);
    z[2 * pair + 1] = radius * __builtin_amdgcn_sinf(b);
  }
}

// ---------------------------------------------------------------------------
// Per-set constants the step needs, loaded into registers.

struct ParF64 {
  double gamma0, dgamma, dt, alpha, V0, sigma, th;
};

struct ParF32 {
  double gamma0, dgamma, th;
  float h, damp, hV0, sigma, V0, th_near;
};

__device__ __forceinline__ ParF64 load_par_f64(const SetDev& s) {
  return ParF64{s.gamma0, s.dgamma, s.dt, s.alpha, s.V0, s.sigma, s.th};
}

__device__ __forceinline__ ParF32 load_par_f32(const SetDev& s) {
  return ParF32{s.gamma0, s.dgamma, s.th, s.h_f, s.damp_f,
                s.hV0_f, s.sigma_f, s.V0_f, s.th_near_f};
}

// ---------------------------------------------------------------------------
// One Euler-Maruyama step k with normal r.
//
// FP64 underdamped, literally Algorithm 1 with the bias of Algorithm 3:
//   phi_k = phi + dt v;  v_k = v + dt (-alpha v - V0 sin phi + V0 gamma_k)
//   + sigma r, where phi, v are the step-(k-1) values and
//   gamma_k = gamma0 + dgamma k.
__device__ __forceinline__ void step_f64_under(const ParF64& p, double kd,
                                               double r, double& phi,
                                               double& v) {
  const double gamma_k = p.gamma0 + p.dgamma * kd;
  const double phi_new = phi + p.dt * v;
  const double force = -p.alpha * v - p.V0 * sin(phi) + p.V0 * gamma_k;
  v = v + p.dt * force + p.sigma * r;
  phi = phi_new;
}

// FP64 overdamped: phi_k = phi + dt (-V0 sin phi + gamma_k) + sigma r.
__device__ __forceinline__ void step_f64_over(const ParF64& p, double kd,
                                              double r, double& phi) {
  const double gamma_k = p.gamma0 + p.dgamma * kd;
  const double drift = -p.V0 * sin(phi) + gamma_k;
  phi = phi + p.dt * drift + p.sigma * r;
}

// FP32C underdamped.  The phase is the compensated pair (phi, c) with true
// value phi - c (Kahan summation of the increments dt v); gamma_k comes from
// the exact step count in FP64 and is rounded once to FP32.
//   v_k = (1 - h alpha) v + h V0 (gamma_k - sin phi) + sigma r
__device__ __forceinline__ void step_f32_under(const ParF32& p, double kd,
                                               float r, float& phi, float& c,
                                               float& v) {
  const float gamma_k = (float)__builtin_fma(p.dgamma, kd, p.gamma0);
  const float s = __builtin_amdgcn_sinf(phi * 0.15915494309189535f);
  // Kahan: y = h v - c; t = phi + y; c = (t - phi) - y; phi = t
  const float y = __builtin_fmaf(p.h, v, -c);
  const float t = phi + y;
  c = (t - phi) - y;
  phi = t;
  const float kick = __builtin_fmaf(p.sigma, r, p.damp * v);
  v = __builtin_fmaf(p.hV0, gamma_k - s, kick);
}

// FP32C overdamped: the increment y = h (gamma_k - V0 sin phi) + sigma r is
// added to the compensated phase (phi, c).
__device__ __forceinline__ void step_f32_over(const ParF32& p, double kd,
                                              float r, float& phi, float& c) {
  const float gamma_k = (float)__builtin_fma(p.dgamma, kd, p.gamma0);
  const float s = __builtin_amdgcn_sinf(phi * 0.15915494309189535f);
  const float drift = __builtin_fmaf(-p.V0, s, gamma_k);
  const float y = __builtin_fmaf(p.h, drift, __builtin_fmaf(p.sigma, r, -c));
  const float t = phi + y;
  c = (t - phi) - y;
  phi = t;
}

// Test of the compensated phase against the FP64 threshold: phi - c formed
// in FP64 holds the compensated value to FP64 rounding (exactly whenever c is
// within 2^-29 of phi's magnitude, the usual case after a Kahan update).
__device__ __forceinline__ bool above_f64(float phi, float c, double th) {
  return ((double)phi - (double)c) > th;
}

}  // namespace fpt
