// mt19937.hpp -- Algorithm 2's generator on gfx950: one MT19937 per replica,
// its 624-word state resident in device memory.
//
// The paper keeps the state of each thread in local memory and regenerates
// all 624 words at once every 624 draws.  Here a lane regenerates the words
// lazily, 4 at a time, in the order the bulk regeneration would: word i of the
// next generation depends on words i and i+1 and on word i+397 (mod 624) as
// they stand in memory at that moment, which is exactly what the in-place
// bulk loop sees.  So the draws are identical to the reference generator, and
// a 4-step block costs one 16-byte store and two 16-byte loads per lane
// instead of a 2.5 KB sweep every 156 blocks.  The loads run two blocks
// ahead of their use, so that enough state is in flight to keep HBM busy.
//
// Layout (structure of arrays, coalesced over a wavefront): group g of the
// state (words 4g .. 4g+3) of slot s is the uint4 at st[g * n_slots + s].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_math.hpp"

namespace fpt {

constexpr uint32_t kMtWords = 624;
constexpr uint32_t kMtGroups = kMtWords / 4;  // 156
constexpr uint32_t kMtFar = 99;               // word 397 = 4 * 99 + 1

// Registers carried from block to block: the group being regenerated and
// the next one (as they stand in memory), and the groups holding words
// i+396 .. i+399 and i+400 .. i+403.
struct MtCarry {
  uint4 cur, nxt;
  uint4 far, far1;
  uint32_t g;  // group of the next block, j mod 156
};

__host__ __device__ __forceinline__ uint32_t mt_group(uint32_t g) {
  return g < kMtGroups ? g : g - kMtGroups;
}

// Standard initialization: w0 = seed, w_i = 1812433253 (w_{i-1} ^ (w_{i-1} >> 30)) + i.
__host__ __device__ inline void mt_seed_slot(uint4* st, uint64_t n_slots, uint64_t slot,
                                    uint32_t seed) {
  uint32_t x = seed;
  uint32_t i = 0;
#pragma unroll 1
  for (uint32_t g = 0; g < kMtGroups; ++g) {
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (i > 0) x = 1812433253u * (x ^ (x >> 30)) + i;
      w[t] = x;
      ++i;
    }
    st[(uint64_t)g * n_slots + slot] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Carry registers for the block with group index g = j mod 156.
__host__ __device__ __forceinline__ MtCarry mt_load(const uint4* st, uint64_t n_slots,
                                                   uint64_t slot, uint32_t g) {
  MtCarry c;
  c.g = g;
  c.cur = st[(uint64_t)g * n_slots + slot];
  c.nxt = st[(uint64_t)mt_group(g + 1) * n_slots + slot];
  c.far = st[(uint64_t)mt_group(g + kMtFar) * n_slots + slot];
  c.far1 = st[(uint64_t)mt_group(g + kMtFar + 1) * n_slots + slot];
  return c;
}

__host__ __device__ __forceinline__ uint32_t mt_next_word(uint32_t lo_src, uint32_t hi_src,
                                                 uint32_t far) {
  // upper bit of word i, lower 31 bits of word i+1
  const uint32_t y = (lo_src & 0x80000000u) | (hi_src & 0x7fffffffu);
  const uint32_t mag = (uint32_t)(-(int32_t)(y & 1u)) & 0x9908b0dfu;
  return far ^ (y >> 1) ^ mag;
}

__host__ __device__ __forceinline__ uint32_t mt_temper(uint32_t y) {
  y ^= y >> 11;
  y ^= (y << 7) & 0x9d2c5680u;
  y ^= (y << 15) & 0xefc60000u;
  y ^= y >> 18;
  return y;
}

// The 4 draws of one block: regenerate group c.g in memory and advance the
// carry by one group.  The groups loaded here (g+2 and g+101) are used one
// and two blocks later; neither is written in between (only g and g+1 are).
__host__ __device__ __forceinline__ Words mt_block(uint4* st, uint64_t n_slots, uint64_t slot,
                                                  MtCarry& c) {
  const uint4 nxt2 = st[(uint64_t)mt_group(c.g + 2) * n_slots + slot];
  const uint4 far2 = st[(uint64_t)mt_group(c.g + kMtFar + 2) * n_slots + slot];
  uint4 n;
  n.x = mt_next_word(c.cur.x, c.cur.y, c.far.y);
  n.y = mt_next_word(c.cur.y, c.cur.z, c.far.z);
  n.z = mt_next_word(c.cur.z, c.cur.w, c.far.w);
  n.w = mt_next_word(c.cur.w, c.nxt.x, c.far1.x);
  st[(uint64_t)c.g * n_slots + slot] = n;
  c.cur = c.nxt;
  c.nxt = nxt2;
  c.far = c.far1;
  c.far1 = far2;
  c.g = mt_group(c.g + 1);
  Words w;
  w.w0 = mt_temper(n.x);
  w.w1 = mt_temper(n.y);
  w.w2 = mt_temper(n.z);
  w.w3 = mt_temper(n.w);
  return w;
}

// Seed of replica `idx` of a set seeded with `seed` (Sect. III.B: the base
// seed plus the replica's index, taken modulo 2^32).
__host__ __device__ __forceinline__ uint32_t mt_replica_seed(uint64_t seed, uint64_t idx) {
  return (uint32_t)(seed + idx);
}

}  // namespace fpt
