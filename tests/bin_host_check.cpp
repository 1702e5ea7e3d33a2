// Host build of the library's histogram binning (device_math.hpp): reads
// lines "k n_bins k_hist" and prints the bin; tests/test_bin_host.py
// compares with exact integer division.
#include <cstdio>

#include "../paper_1802_05065_amd/csrc/device_math.hpp"

int main() {
  long long k, kh;
  unsigned nb;
  while (std::scanf("%lld %u %lld", &k, &nb, &kh) == 3)
    std::printf("%u\n", fpt::hist_bin_of(k, nb, kh, (double)nb / (double)kh));
  return 0;
}
