// f64_math.hpp -- double-precision sine / cosine and the Box-Muller log of
// the FP64 integrator, written for the arguments it sees: phases of moderate
// size, angles in (0, 2 pi), uniforms in (0, 1).  No special-case handling
// (NaN and infinities give NaN).  Errors stay within about 2 units in the last
// place of the correctly rounded values (checked on the host against the C
// library by tests/test_f64_math_host.py).
//
// Methods: Cody and Waite's additive reduction by pi (sin) or pi/2 (sin and
// cos together) with the constant split in three parts (W. J. Cody, W.
// Waite, "Software Manual for the Elementary Functions", 1980), the Taylor
// series of sin on [-pi/2, pi/2] and of sin and cos on [-pi/4, pi/4], and
// ln m = 2 atanh((m - 1)/(m + 1)) on [sqrt(2)/2, sqrt(2)) by its odd power
// series.  Coefficients are 1/n! and 1/n rounded to double.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace fpt {
namespace f64m {

constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
// pi/2 = kPio2a + kPio2b + kPio2c to 1e-37; the first two carry 33
// significant bits, so n kPio2a and n kPio2b are exact for |n| < 2^20
constexpr double kPio2a = 0x1.921fb54400000p+0;
constexpr double kPio2b = 0x1.0b4611a600000p-34;
constexpr double kPio2c = 0x1.3198a2e037073p-69;

// ln 2 = kLn2a + kLn2b to 1e-27; kLn2a carries 32 significant bits, so
// e kLn2a is exact for the exponents of (0, 1)
constexpr double kLn2a = 0x1.62e42ff000000p-1;
constexpr double kLn2b = -0x1.718432a1b0e26p-35;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

// One Horner step p z + c as a single three-operand v_fma_f64 with the
// coefficient kept in registers: written as fma(), the compiler turns each
// step into a copy of c plus the two-operand fma that overwrites its addend.
// (Host builds use fma().)
__host__ __device__ __forceinline__ double horner(double p, double z, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(z), "v"(c));
  return r;
#else
  return fma(p, z, c);
#endif
}

// x with its sign flipped when bit 0 of `bits` is set (an xor of the sign
// bit: no select)
__host__ __device__ __forceinline__ double flip_sign(double x, uint32_t bits) {
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) ^ ((uint64_t)(bits & 1u) << 63));
}

// The low bits of an integer-valued double n with |n| < 2^51: n + 1.5 2^52
// lies in [2^52, 2^53), where the significand's last bit is worth 1, and
// holds n in its low bits (two's complement for n < 0)
__host__ __device__ __forceinline__ uint32_t low_bits(double n) {
  return (uint32_t)__builtin_bit_cast(uint64_t, n + 0x1.8p52);
}

// sin r and cos r for |r| <= pi/4 (plus the reduction's slack): Taylor
// polynomials through r^17 and r^16, whose next terms stay below 2^-62 and
// 2^-58 of the result there
__host__ __device__ __forceinline__ void sincos_poly(double r, double& s, double& c) {
  const double z = r * r;
  double ps = 0x1.952c77030ad4ap-49;         //  1/17!
  ps = horner(ps, z, -0x1.ae7f3e733b81fp-41);   // -1/15!
  ps = horner(ps, z, 0x1.6124613a86d09p-33);    //  1/13!
  ps = horner(ps, z, -0x1.ae64567f544e4p-26);   // -1/11!
  ps = horner(ps, z, 0x1.71de3a556c734p-19);    //  1/9!
  ps = horner(ps, z, -0x1.a01a01a01a01ap-13);   // -1/7!
  ps = horner(ps, z, 0x1.1111111111111p-7);     //  1/5!
  ps = horner(ps, z, -0x1.5555555555555p-3);    // -1/3!
  s = fma(r * z, ps, r);
  double pc = 0x1.ae7f3e733b81fp-45;         //  1/16!
  pc = horner(pc, z, -0x1.93974a8c07c9dp-37);   // -1/14!
  pc = horner(pc, z, 0x1.1eed8eff8d898p-29);    //  1/12!
  pc = horner(pc, z, -0x1.27e4fb7789f5cp-22);   // -1/10!
  pc = horner(pc, z, 0x1.a01a01a01a01ap-16);    //  1/8!
  pc = horner(pc, z, -0x1.6c16c16c16c17p-10);   // -1/6!
  pc = horner(pc, z, 0x1.5555555555555p-5);     //  1/4!
  pc = horner(pc, z, -0.5);                     // -1/2!
  c = fma(z, pc, 1.0);
}

// x = q pi/2 + r with |r| <= pi/4 (|x| < 2^20): the first subtraction is
// exact, the other two round once each
__host__ __device__ __forceinline__ double reduce_pio2(double x, int& q) {
  const double n = rint(x * kTwoOverPi);
  double r = fma(-n, kPio2a, x);
  r = fma(-n, kPio2b, r);
  r = fma(-n, kPio2c, r);
  q = (int)n;
  return r;
}

// sin x: x = n pi + r with |r| <= pi/2 (pi split as pi/2 above), sin x =
// (-1)^n sin r, and sin r by its Taylor polynomial through r^21 (next term
// below 2^-59 of the result): one polynomial and no quadrant selection.
// Below 2^20 rad the first reduction step is exact and the result is within
// about 2 ulp; beyond, that step rounds once, and from 2^30 rad on the phase
// is first brought below pi the same way (random phases stay within 2.3 ulp
// up to 2^41 rad, measured; next to multiples of pi the error is absolute,
// far below the phase's own ulp; past 2^52 rad, where the phase's ulp
// exceeds 1, the result means nothing).  No general library routine: one
// beside it costs the integrator registers it then spills.
constexpr double kOneOverPi = 0x1.45f306dc9c883p-2;
constexpr double kPia = 0x1.921fb54400000p+1;
constexpr double kPib = 0x1.0b4611a600000p-33;
constexpr double kPic = 0x1.3198a2e037073p-68;

__host__ __device__ __forceinline__ double sin_f64(double x) {
  if (__builtin_expect(!(fabs(x) < 0x1p30), 0)) {
    // far phases: first take out a multiple of pi the same way (the
    // product exact inside each fma, one rounding per step; the result's
    // absolute error stays far below the phase's own ulp)
    const double m = rint(x * kOneOverPi);
    x = fma(-m, kPic, fma(-m, kPib, fma(-m, kPia, x)));
    x = flip_sign(x, low_bits(m));
  }
  const double n = rint(x * kOneOverPi);
  double r = fma(-n, kPia, x);
  r = fma(-n, kPib, r);
  r = fma(-n, kPic, r);
  const double z = r * r;
  double p = 0x1.71b8ef6dcf572p-66;          //  1/21!
  p = horner(p, z, -0x1.2f49b46814157p-57);     // -1/19!
  p = horner(p, z, 0x1.952c77030ad4ap-49);      //  1/17!
  p = horner(p, z, -0x1.ae7f3e733b81fp-41);     // -1/15!
  p = horner(p, z, 0x1.6124613a86d09p-33);      //  1/13!
  p = horner(p, z, -0x1.ae64567f544e4p-26);     // -1/11!
  p = horner(p, z, 0x1.71de3a556c734p-19);      //  1/9!
  p = horner(p, z, -0x1.a01a01a01a01ap-13);     // -1/7!
  p = horner(p, z, 0x1.1111111111111p-7);       //  1/5!
  p = horner(p, z, -0x1.5555555555555p-3);      // -1/3!
  const double s = fma(r * z, p, r);
  // (-1)^n from n itself (an integer-valued double; no conversion)
  return flip_sign(s, low_bits(n));
}

// Both at once, for |x| < 2^20 only (the Box-Muller angles lie in
// (0, 2 pi)); no fallback.
__host__ __device__ __forceinline__ void sincos_f64(double x, double* s, double* c) {
  int q;
  const double r = reduce_pio2(x, q);
  double ps, pc;
  sincos_poly(r, ps, pc);
  const double vs = (q & 1) ? pc : ps;
  const double vc = (q & 1) ? ps : pc;
  *s = flip_sign(vs, (uint32_t)q >> 1);
  *c = flip_sign(vc, (uint32_t)(q + 1) >> 1);
}

// Reciprocal and square root for the Box-Muller radius, where the operands
// are positive normal numbers of moderate size: the hardware estimate
// (v_rcp_f64 / v_rsq_f64) refined by Newton-Raphson steps, without the
// scaling and special-case handling of the general division and sqrt.
// The hardware estimates are good to about 2^29 ulp, 2^-23 relative.  Host
// builds start from a float estimate pushed off by a further 2^-22, worse
// than the hardware's, so the host check covers the refinement.
__host__ __device__ __forceinline__ double rcp_estimate(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(d);
#else
  return (double)(1.0f / (float)d) * (1.0 + 0x1p-22);
#endif
}

__host__ __device__ __forceinline__ double rsq_estimate(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsq(x);
#else
  return (double)(1.0f / std::sqrt((float)x)) * (1.0 - 0x1p-22);
#endif
}

// n / d for d in [1, 4): two Newton-Raphson steps on 1/d, then the quotient
// corrected once by its residual
__host__ __device__ __forceinline__ double div_moderate(double n, double d) {
  double y = rcp_estimate(d);
  double e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  const double q = n * y;
  return fma(fma(-q, d, n), y, q);
}

// sqrt(x) for normal x > 0: from r ~ 1/sqrt(x), g = x r and h = r/2 refined
// together (Goldschmidt), then g corrected by its residual, twice
__host__ __device__ __forceinline__ double sqrt_positive(double x) {
  const double r = rsq_estimate(x);
  double g = x * r;
  double h = 0.5 * r;
  const double t = fma(-g, h, 0.5);
  g = fma(g, t, g);
  h = fma(h, t, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// -2 ln a for a normal number in (0, 1]: a = m 2^e with m in
// [sqrt(2)/2, sqrt(2)), ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^21/21)
// with s = (m - 1)/(m + 1), |s| <= 0.172 (next term below 2^-60 of ln m)
__host__ __device__ __forceinline__ double minus_two_log(double a) {
  int e;
  double m = frexp(a, &e);
  if (m < kSqrtHalf) {
    m = 2.0 * m;
    --e;
  }
  const double s = div_moderate(m - 1.0, m + 1.0);
  const double z = s * s;
  double p = 0x1.8618618618618p-5;   // 1/21
  p = horner(p, z, 0x1.af286bca1af28p-5);  // 1/19
  p = horner(p, z, 0x1.e1e1e1e1e1e1ep-5);  // 1/17
  p = horner(p, z, 0x1.1111111111111p-4);  // 1/15
  p = horner(p, z, 0x1.3b13b13b13b14p-4);  // 1/13
  p = horner(p, z, 0x1.745d1745d1746p-4);  // 1/11
  p = horner(p, z, 0x1.c71c71c71c71cp-4);  // 1/9
  p = horner(p, z, 0x1.2492492492492p-3);  // 1/7
  p = horner(p, z, 0x1.999999999999ap-3);  // 1/5
  p = horner(p, z, 0x1.5555555555555p-2);  // 1/3
  const double t = 2.0 * s;
  const double de = (double)e;
  // ln a = e ln2 + t + t z p, the small parts summed first
  const double lo = fma(de, kLn2b, (t * z) * p);
  const double ln_a = fma(de, kLn2a, t + lo);
  return -2.0 * ln_a;
}

}  // namespace f64m
}  // namespace fpt
