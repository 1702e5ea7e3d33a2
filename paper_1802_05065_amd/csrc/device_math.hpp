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

#include "f64_math.hpp"
#include "internal.hpp"

namespace fpt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The 32x32 -> 64
// products map to v_mad_u64_u32, the XOR pairs to gfx950's v_bitop3_b32; with
// a wave-uniform key the key schedule lives in scalar registers.
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
    // three-input XOR in one v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// The same with a wavefront-uniform key: each round key is formed on the
// scalar unit just before its round (the opaque copy stops the compiler from
// hoisting all 20 into scalar registers at once, which would cost the
// integrator a resident wave).  Round 0's product of the replica index is
// the same for every block, but forming it here keeps the two product
// chains of each round independent, which the scheduler interleaves; passed
// in precomputed, it offsets the chains and the loop ran 5% slower.
__device__ __forceinline__ Words philox4x32_10_uniform_key(uint32_t c0, uint32_t c1,
                                                           uint32_t c2, uint32_t c3,
                                                           uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    asm volatile("" : "+s"(k0), "+s"(k1));
    const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// The generator for a counter whose words 1-3 stay fixed while word 0 (the
// block index's low half) steps: a replica's blocks between two crossings
// of a multiple of 2^32.  Of rounds 0 and 1, every part that does not
// depend on word 0 is formed once (round 0's product of word 2 and the
// new word 0 it gives, round 1's product of that word, and the words and
// key XORs they meet); what is left of the two rounds is 2 products and 3
// two-input XORs instead of 4 products and 4 three-input XORs.  The words
// equal philox4x32_10's bit for bit (host-checked against the oracle's).
// M0 = 0xD2511F53 and M1 = 0xCD9E8D57 are the round multipliers, W0 =
// 0x9E3779B9 and W1 = 0xBB67AE85 the key increments.
struct PhiloxFixed {
  uint32_t b;  // c3 ^ k1: round 0's second XOR without hi(M0 c0)
  uint32_t d;  // lo(M1 c2) ^ (k0 + W0): round 1's first XOR without its product
  uint32_t e;  // hi(M0 A) ^ (k1 + W1): round 1's second XOR without lo(M0 c0)
  uint32_t f;  // lo(M0 A): round 1's new word 3
};

__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

// (A = hi(M1 c2) ^ c1 ^ k0 is round 0's new word 0.)
__host__ __device__ __forceinline__ PhiloxFixed philox_fixed_part(uint32_t c1, uint32_t c2,
                                                                  uint32_t c3, uint32_t k0,
                                                                  uint32_t k1) {
  const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
  const uint32_t A = xor3((uint32_t)(pb >> 32), c1, k0);
  const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)A;
  PhiloxFixed f;
  f.b = c3 ^ k1;
  f.d = (uint32_t)pb ^ (k0 + 0x9E3779B9u);
  f.e = (uint32_t)(pa >> 32) ^ (k1 + 0xBB67AE85u);
  f.f = (uint32_t)pa;
  return f;
}

// philox4x32_10(c0, c1, c2, c3, k0, k1) given philox_fixed_part(c1, c2, c3,
// k0, k1); the key is wavefront-uniform as in philox4x32_10_uniform_key.
__host__ __device__ __forceinline__ Words philox4x32_10_fixed(uint32_t c0,
                                                              const PhiloxFixed& f,
                                                              uint32_t k0, uint32_t k1) {
  // round 0: only the product of word 0 varies
  const uint64_t pa0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
  const uint32_t n2 = (uint32_t)(pa0 >> 32) ^ f.b;
  // round 1: only the product of the new word 2 varies
  const uint64_t pb1 = (uint64_t)0xCD9E8D57u * (uint64_t)n2;
  c0 = (uint32_t)(pb1 >> 32) ^ f.d;
  uint32_t c1 = (uint32_t)pb1;
  uint32_t c2 = (uint32_t)pa0 ^ f.e;
  uint32_t c3 = f.f;
  // (formed in the loop on the scalar unit, not held across it: two more
  // live scalar registers cost the FP32C kernel its eighth resident wave)
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(k0), "+s"(k1));
#endif
  k0 += 2u * 0x9E3779B9u;
  k1 += 2u * 0xBB67AE85u;
#pragma unroll
  for (int round = 2; round < 10; ++round) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(k0), "+s"(k1));
#endif
    const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
    const uint32_t m2 = xor3((uint32_t)(pa >> 32), c3, k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = m2;
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
    const double radius = f64m::sqrt_positive(f64m::minus_two_log(a));
    const double angle = 2.0 * kPi * b;
    double s, c;
    f64m::sincos_f64(angle, &s, &c);
    z[2 * pair] = radius * c;
    z[2 * pair + 1] = radius * s;
  }
}

// FP32: hardware transcendentals.  v_log_f32 is log2 and v_sin/v_cos_f32 take
// their argument in revolutions, so 2 pi b needs no multiply.  The integrator
// uses the pair in factored form: radius' = sqrt(-log2 a) and the angle's
// cos / sin, with the constant sqrt(2 ln 2) folded into its noise scale, so
// z = sqrt(2 ln 2) radius' (cos, sin).
constexpr float kSqrt2Ln2 = 1.1774100225154747f;

struct BoxMullerF32 {
  float radius[2];  // sqrt(-log2 a) of pairs (w0, w1) and (w2, w3)
  float c[2], s[2];
};

__device__ __forceinline__ BoxMullerF32 box_muller_f32(const Words& w) {
  const uint32_t x[4] = {w.w0, w.w1, w.w2, w.w3};
  BoxMullerF32 bm;
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const float a = __builtin_fmaf((float)x[2 * pair], 0x1p-32f, 0x1p-33f);
    // angle: 1 + (x >> 9) 2^-23 in [1, 2) revolutions in one v_alignbit_b32
    // (the 23 leading bits of x as the mantissa of a float with exponent 0);
    // sin and cos have period 1 in revolutions
    const float b = __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x[2 * pair + 1], 9));
    bm.radius[pair] = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(a));
    bm.c[pair] = __builtin_amdgcn_cosf(b);
    bm.s[pair] = __builtin_amdgcn_sinf(b);
  }
  return bm;
}

// The four standard normals of a block in FP32 (diagnostics).
__device__ __forceinline__ void normals_f32(const Words& w, float z[4]) {
  const BoxMullerF32 bm = box_muller_f32(w);
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const float r = kSqrt2Ln2 * bm.radius[pair];
    z[2 * pair] = r * bm.c[pair];
    z[2 * pair + 1] = r * bm.s[pair];
  }
}

// ---------------------------------------------------------------------------
// Per-set constants the step needs, loaded into registers.

struct ParF64 {
  double gamma0, dgamma, dt, alpha, V0, sigma, th;
};

// FP32C constants, phase in revolutions (phi / 2 pi):
//   underdamped  v_k = damp v + G_k + nkS sin(2 pi phr) + sig z_k,
//                phr_k = phr + h_rev v
//   overdamped   phr_k = phr + G_k + nkS sin(2 pi phr) + sig z_k
// (the phase sum compensated once per block of 4 steps, see below)
// with G_k = gA + gB k evaluated in FP64 from the exact step k, nkS = -kS,
// and dG, dG2, dG3 the bias offsets of a block's steps 2, 3, 4 from its first.
struct ParF32 {
  double gA, gB, th_rev;
  float h_rev, damp, nkS, sig, dG, dG2, dG3, th_near_rev;
};

__device__ __forceinline__ ParF64 load_par_f64(const SetDev& s) {
  return ParF64{s.gamma0, s.dgamma, s.dt, s.alpha, s.V0, s.sigma, s.th};
}

__device__ __forceinline__ ParF32 load_par_f32(const SetDev& s) {
  return ParF32{s.gA, s.gB, s.th_rev, s.h_rev_f, s.damp_f, s.nkS_f, s.sig_f, s.dG_f,
                s.dG2_f, s.dG3_f, s.th_near_rev_f};
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
  const double force = -p.alpha * v - p.V0 * f64m::sin_f64(phi) + p.V0 * gamma_k;
  v = v + p.dt * force + p.sigma * r;
  phi = phi_new;
}

// FP64 underdamped, semi-implicit (symplectic) Euler: v_k as above, then
// phi_k = phi + dt v_k.
__device__ __forceinline__ void step_f64_under_si(const ParF64& p, double kd,
                                                  double r, double& phi,
                                                  double& v) {
  const double gamma_k = p.gamma0 + p.dgamma * kd;
  const double force = -p.alpha * v - p.V0 * f64m::sin_f64(phi) + p.V0 * gamma_k;
  v = v + p.dt * force + p.sigma * r;
  phi = phi + p.dt * v;
}

// FP64 overdamped: phi_k = phi + dt (-V0 sin phi + gamma_k) + sigma r.
__device__ __forceinline__ void step_f64_over(const ParF64& p, double kd,
                                              double r, double& phi) {
  const double gamma_k = p.gamma0 + p.dgamma * kd;
  const double drift = -p.V0 * f64m::sin_f64(phi) + gamma_k;
  phi = phi + p.dt * drift + p.sigma * r;
}

// FP32C steps.  Between blocks the phase is the compensated pair (phr, e)
// in revolutions, true value phr + e.  Inside a block of 4 steps a plain
// FP32 running sum d starts at e and takes the steps' increments (at most
// 4 of them, so its own rounding stays far below one increment's noise);
// step q+1 sees the phase x_q = phr + d_q, rounded once, and the block's
// end splits phr + d_4 into the new pair with the error term of the
// rounded sum (Fast2Sum: |phr| >= |d| near any threshold).  `a` enters as
// G_k rounded to FP32 and is consumed; `zs` is the noise factor
// sig*radius' and `trig` the cos or sin of the pair's angle.  Each update
// is a multiply-add into a value that dies with it, so the compiler can use
// the two-operand v_fmac_f32, which issues at twice the rate of the
// three-operand v_fma_f32 on gfx950.

// Underdamped, explicit (Algorithm 1): the phase advance uses the old
// velocity.
__device__ __forceinline__ void step_f32_under(const ParF32& p, float a, float zs,
                                               float trig, float x, float& d, float& v) {
  const float s = __builtin_amdgcn_sinf(x);
  d = __builtin_fmaf(p.h_rev, v, d);
  a = __builtin_fmaf(zs, trig, a);
  a = __builtin_fmaf(p.nkS, s, a);
  v = __builtin_fmaf(p.damp, v, a);
}

// Underdamped, semi-implicit: the velocity first, then the phase moves with
// the new velocity.
__device__ __forceinline__ void step_f32_under_si(const ParF32& p, float a, float zs,
                                                  float trig, float x, float& d,
                                                  float& v) {
  const float s = __builtin_amdgcn_sinf(x);
  a = __builtin_fmaf(zs, trig, a);
  a = __builtin_fmaf(p.nkS, s, a);
  v = __builtin_fmaf(p.damp, v, a);
  d = __builtin_fmaf(p.h_rev, v, d);
}

// Overdamped: the increment G_k - kS sin(2 pi x) + sig z_k joins the
// running sum.
__device__ __forceinline__ void step_f32_over(const ParF32& p, float a, float zs,
                                              float trig, float x, float& d) {
  const float s = __builtin_amdgcn_sinf(x);
  a = __builtin_fmaf(zs, trig, a);
  a = __builtin_fmaf(p.nkS, s, a);
  d = d + a;
}

// End of a block: phr + d becomes the pair (phr', e') with phr' = phr + d
// rounded and e' = d - (phr' - phr), the part of d that phr' lost.
__device__ __forceinline__ void fold_advance(float d, float& phr, float& e) {
  const float t = phr + d;
  e = d - (t - phr);
  phr = t;
}

// Bias terms G_k of a block's 4 steps: the first from the exact step count
// k1 = 4 j + 1 in FP64, the others by FP32 offsets.
struct BlockG {
  float g[4];
};

__device__ __forceinline__ BlockG block_g4(const ParF32& p, double k1, double gA) {
  BlockG b;
  b.g[0] = (float)__builtin_fma(p.gB, k1, gA);
  b.g[1] = b.g[0] + p.dG;
  b.g[2] = b.g[0] + p.dG2;
  b.g[3] = b.g[0] + p.dG3;
  return b;
}

// Histogram bin of escape step k in [1, k_hist]: floor((k-1) n_bins / k_hist),
// exactly, with scale = n_bins / k_hist.  The FP64 quotient is within 1e-12
// of the true one (k-1 < 2^53, quotient < 2^12), so one integer correction
// step either way makes it exact; a software 64-bit division here would set
// the integrator's register count.
__host__ __device__ __forceinline__ uint32_t hist_bin_of(int64_t k, uint32_t n_bins,
                                                         int64_t k_hist, double scale) {
  const uint64_t num = (uint64_t)(k - 1) * (uint64_t)n_bins;
  const uint64_t kh = (uint64_t)k_hist;
  const double est = (double)(k - 1) * scale;
  uint32_t b = est < (double)(n_bins - 1) ? (uint32_t)est : n_bins - 1;
  if (b > 0 && (uint64_t)b * kh > num) --b;
  if ((uint64_t)(b + 1) * kh <= num) ++b;
  return b;
}

// Test of the compensated phase against the FP64 threshold (revolutions):
// phr + e formed in FP64 holds the compensated value to FP64 rounding.
__device__ __forceinline__ bool above_f64(float phr, float e, double th_rev) {
  return ((double)phr + (double)e) > th_rev;
}

}  // namespace fpt
