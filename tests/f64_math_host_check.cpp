// Host build of the FP64 integrator's sine / cosine / log (csrc/f64_math.hpp)
// against the C library's long-double functions: prints, per function and
// argument range, the largest error in units of the last place of the
// double result.  tests/test_f64_math_host.py runs it and holds the bounds.
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../paper_1802_05065_amd/csrc/f64_math.hpp"

namespace {

uint64_t g_state = 0x243F6A8885A308D3ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform(double lo, double hi) {
  return lo + (hi - lo) * ((double)(next_u64() >> 11) * 0x1p-53);
}

// error of `got` against the exact value `ref` in units of the last place
// of the double nearest to ref
double ulps(double got, long double ref) {
  const double r = (double)ref;
  if (r == 0.0) return got == 0.0 ? 0.0 : 1e300;
  int e;
  std::frexp(r, &e);
  const long double ulp = std::ldexp(1.0L, e - 53);
  return (double)(std::fabs((long double)got - ref) / ulp);
}

struct Worst {
  double err = 0.0, arg = 0.0;
  void add(double e, double x) {
    if (e > err) {
      err = e;
      arg = x;
    }
  }
};

void report(const char* name, const Worst& w, long n) {
  std::printf("%s %ld %.4f %a\n", name, n, w.err, w.arg);
}

}  // namespace

int main(int argc, char** argv) {
  const long n = argc > 1 ? atol(argv[1]) : 2000000;
  // sin of phases: moderate arguments, and points next to multiples of pi/2
  {
    Worst w;
    for (long i = 0; i < n; ++i) {
      const double x = uniform(-40.0, 40.0);
      w.add(ulps(fpt::f64m::sin_f64(x), std::sin((long double)x)), x);
    }
    report("sin_moderate", w, n);
    Worst z;
    for (long i = 0; i < n; ++i) {
      const long k = (long)(next_u64() % 64) - 32;
      const double x = (double)k * 1.5707963267948966 + uniform(-1e-6, 1e-6);
      z.add(ulps(fpt::f64m::sin_f64(x), std::sin((long double)x)), x);
    }
    report("sin_near_zeros", z, n);
    Worst b;
    for (long i = 0; i < n / 4; ++i) {
      const double x = uniform(-1e6, 1e6);
      b.add(ulps(fpt::f64m::sin_f64(x), std::sin((long double)x)), x);
    }
    report("sin_large", b, n / 4);
    Worst f;
    for (long i = 0; i < n / 4; ++i) {
      const double x = std::ldexp(uniform(1.0, 2.0), 30 + (int)(next_u64() % 11));
      f.add(ulps(fpt::f64m::sin_f64(x), std::sin((long double)x)), x);
    }
    report("sin_far", f, n / 4);
  }
  // sin and cos of Box-Muller angles 2 pi b, b = (x + 1/2) 2^-32
  {
    Worst ws, wc;
    const double two_pi = 2.0 * 3.14159265358979323846;
    for (long i = 0; i < n; ++i) {
      const uint32_t x = (uint32_t)next_u64();
      const double b = ((double)x + 0.5) * 0x1p-32;
      const double angle = two_pi * b;
      double s, c;
      fpt::f64m::sincos_f64(angle, &s, &c);
      ws.add(ulps(s, std::sin((long double)angle)), angle);
      wc.add(ulps(c, std::cos((long double)angle)), angle);
    }
    report("sincos_angle_sin", ws, n);
    report("sincos_angle_cos", wc, n);
  }
  // -2 ln a over the uniforms, including both ends
  {
    Worst w;
    for (long i = 0; i < n; ++i) {
      uint32_t x = (uint32_t)next_u64();
      if (i < 64) x = (uint32_t)i;
      if (i >= 64 && i < 128) x = 0xFFFFFFFFu - (uint32_t)(i - 64);
      const double a = ((double)x + 0.5) * 0x1p-32;
      w.add(ulps(fpt::f64m::minus_two_log(a), -2.0L * std::log((long double)a)), a);
    }
    report("minus_two_log", w, n);
    Worst r;
    for (long i = 0; i < n; ++i) {
      uint32_t x = (uint32_t)next_u64();
      if (i < 64) x = (uint32_t)i;
      if (i >= 64 && i < 128) x = 0xFFFFFFFFu - (uint32_t)(i - 64);
      const double a = ((double)x + 0.5) * 0x1p-32;
      const double l = fpt::f64m::minus_two_log(a);
      r.add(ulps(fpt::f64m::sqrt_positive(l), std::sqrt((long double)l)), l);
    }
    report("radius_sqrt", r, n);
  }
  return 0;
}
