// Host build of the generator variant for fixed counter words 1-3
// (device_math.hpp: philox_fixed_part + philox4x32_10_fixed): reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four words; tests/test_philox_fixed.py
// compares them with the oracle's Philox4x32-10.
#include <cstdio>

#include "../paper_1802_05065_amd/csrc/device_math.hpp"

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const fpt::PhiloxFixed f = fpt::philox_fixed_part(c1, c2, c3, k0, k1);
    const fpt::Words w = fpt::philox4x32_10_fixed(c0, f, k0, k1);
    std::printf("%u %u %u %u\n", w.w0, w.w1, w.w2, w.w3);
  }
  return 0;
}
