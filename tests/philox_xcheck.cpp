// Cross-check harness: prints Philox4x32-10 words computed by PyTorch's
// header-only at::philox_engine, an implementation independent of the oracle.
// stdin: lines "seed subsequence offset"; stdout: 4 hex words per line.
// philox_engine(seed, subsequence, offset) uses key = (seed lo, seed hi) and
// counter = (offset lo, offset hi, subsequence lo, subsequence hi), which is
// the (seed, replica, block) layout of the oracle's generator.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cinttypes>
#include <cstdio>

int main() {
  unsigned long long seed, subseq, offset;
  while (std::scanf("%llu %llu %llu", &seed, &subseq, &offset) == 3) {
    at::philox_engine eng(seed, subseq, offset);
    uint32_t w[4];
    for (int i = 0; i < 4; ++i) w[i] = eng();
    std::printf("%08" PRIx32 " %08" PRIx32 " %08" PRIx32 " %08" PRIx32 "\n", w[0], w[1],
                w[2], w[3]);
  }
  return 0;
}
