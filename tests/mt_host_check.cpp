// Host build of the library's lazily regenerated MT19937 (mt19937.hpp): three
// interleaved slots, the carry reloaded every 37 blocks as a launch restore
// does.  Prints 4 words per slot and block; tests/test_mt_host.py compares
// them with the oracle's generator.
#include <cstdio>
#include <vector>

#include "../paper_1802_05065_amd/csrc/mt19937.hpp"
using namespace fpt;
int main() {
  const uint64_t n_slots = 3;
  std::vector<uint4> st(156 * n_slots);
  uint32_t seeds[3] = {5489u, 5490u, 4294967295u};
  MtCarry c[3];
  for (int s = 0; s < 3; ++s) { mt_seed_slot(st.data(), n_slots, s, seeds[s]); c[s] = mt_load(st.data(), n_slots, s, 0); }
  for (int b = 0; b < 400; ++b)
    for (int s = 0; s < 3; ++s) {
      if (b % 37 == 0) c[s] = mt_load(st.data(), n_slots, s, (uint32_t)(b % 156));
      Words w = mt_block(st.data(), n_slots, s, c[s]);
      printf("%u %u %u %u\n", w.w0, w.w1, w.w2, w.w3);
    }
}
