// kernels.hip -- gfx950 kernels of the first-passage-time library.
//
// The integrator is one kernel template: one wavefront lane holds R replicas
// ("slots") in registers and advances them in blocks of 4 Euler steps (one
// Philox call feeds the 4 normals of a block).  A launch runs at most
// `blocks` blocks and leaves every slot's state resident in device memory, so
// long runs are split into launches and a server can add work between them.
//
// Scheduling (Sect. III.B, the streaming figure): with `refill` set, a slot
// whose replica escaped or was censored takes the next undrawn replica from a
// global cursor.  The wavefront draws for all its free slots with one atomic
// (ballot + popcount + mbcnt), so uneven escape times do not idle lanes.
// Without `refill` each slot keeps the replica assigned at the start
// (one realization per thread, Algorithm 1's launch).
//
// Several parameter sets: a wavefront integrates a block for the lanes of
// one set at a time, with that set's constants and Philox key in scalar
// registers.  Multi-set refill runs keep wavefronts to one set: between
// launches the active slots are sorted by set (each set starting a
// wavefront) and the free slots refilled in queue order, and inside a launch
// only a wavefront free in every lane draws (64 replicas, one chunk of one
// set); such a wavefront runs its blocks with the constants fixed.
//
// With MT set the words of a block come from the replica's own MT19937
// (Algorithm 2), whose state stays in device memory (mt19937.hpp); a slot
// seeds it when it takes a new replica.
//
// Results (the escape-time / switching-current histograms of Sect. II.B and
// IV.B): finished replicas write their step to the caller's array, then add
// to a per-workgroup LDS hash table of (set, bin) counts and of per-set
// integer moments; lanes of a wavefront that finish in the same block with
// the same (set, bin) are merged first.  At the end of a launch each
// workgroup adds its LDS tables to the global histogram / moments with one
// atomic per occupied entry.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_math.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "mt19937.hpp"

namespace fpt {

// ---------------------------------------------------------------------------
// Slot state

template <bool FP64>
struct Slot;

template <>
struct Slot<true> {
  uint32_t set;
  uint64_t idx, j;
  double kd;  // 4 j + 1, the step number of the block's first step (exact)
  double phi, v;
  float e;    // unused in FP64
};

template <>
struct Slot<false> {
  uint32_t set;
  uint64_t idx, j;
  double kd;
  float phi, v;  // phi: phase in revolutions
  float e;       // its error term: true phase = phi + e (between blocks)
};

// Constants of one set that the block loop reads, held in scalar registers:
// a wavefront integrates a block for lanes of one set at a time.
template <bool FP64>
struct SetPar;

template <>
struct SetPar<true> {
  ParF64 p;
  uint32_t k0, k1;  // Philox key: the set's seed
};

template <>
struct SetPar<false> {
  ParF32 p;
  uint32_t k0, k1;
};

// The set table does not change while a launch runs; read through the
// constant address space, a wavefront-uniform set index gives scalar loads.
using ConstSetDev = const __attribute__((address_space(4))) SetDev;

template <bool FP64>
__device__ __forceinline__ SetPar<FP64> load_setpar(const SetDev* sets, uint32_t set) {
  const ConstSetDev& d = ((ConstSetDev*)sets)[set];
  SetPar<FP64> P;
  if constexpr (FP64) {
    P.p = ParF64{d.gamma0, d.dgamma, d.dt, d.alpha, d.V0, d.sigma, d.th};
  } else {
    P.p = ParF32{d.gA, d.gB, d.th_rev, d.h_rev_f, d.damp_f, d.nkS_f, d.sig_f, d.dG_f,
                 d.dG2_f, d.dG3_f, d.th_near_rev_f};
  }
  const uint64_t seed = d.seed;
  P.k0 = (uint32_t)seed;
  P.k1 = (uint32_t)(seed >> 32);
  return P;
}

template <bool FP64>
__device__ __forceinline__ void start_replica(Slot<FP64>& s, uint32_t set,
                                              uint64_t idx, const SetDev& sd) {
  s.set = set;
  s.idx = idx;
  s.j = 0;
  s.kd = 1.0;
  if constexpr (FP64) {
    s.phi = sd.phi0;
    s.v = sd.v0;
    s.e = 0.0f;
  } else {
    s.phi = sd.phr0_f;
    s.e = sd.e0_f;
    s.v = sd.v0_f;
  }
}

// Resident-state encoding: st_phi holds the FP64 phase, or the FP32 pair
// (phi, e) in the low / high word; st_v the FP64 or FP32 velocity.
template <bool FP64>
__device__ __forceinline__ void store_slot(const SliceArgs& a, uint64_t slot,
                                           const Slot<FP64>& s) {
  a.st_set[slot] = s.set;
  if (s.set == kInactive) return;
  a.st_idx[slot] = s.idx;
  a.st_j[slot] = s.j;
  if constexpr (FP64) {
    a.st_phi[slot] = (unsigned long long)__double_as_longlong(s.phi);
    a.st_v[slot] = (unsigned long long)__double_as_longlong(s.v);
  } else {
    a.st_phi[slot] = (unsigned long long)__float_as_uint(s.phi) |
                     ((unsigned long long)__float_as_uint(s.e) << 32);
    a.st_v[slot] = (unsigned long long)__float_as_uint(s.v);
  }
}

template <bool FP64>
__device__ __forceinline__ void restore_slot(const SliceArgs& a, uint64_t slot,
                                             Slot<FP64>& s) {
  s.set = a.st_set[slot];
  s.idx = 0;
  s.j = 0;
  s.kd = 0.0;
  s.phi = 0;
  s.v = 0;
  s.e = 0.0f;
  if (s.set == kInactive) return;
  s.idx = a.st_idx[slot];
  s.j = a.st_j[slot];
  s.kd = 4.0 * (double)s.j + 1.0;
  const unsigned long long ph = a.st_phi[slot];
  const unsigned long long vv = a.st_v[slot];
  if constexpr (FP64) {
    s.phi = __longlong_as_double((long long)ph);
    s.v = __longlong_as_double((long long)vv);
    s.e = 0.0f;
  } else {
    s.phi = __uint_as_float((uint32_t)ph);
    s.e = __uint_as_float((uint32_t)(ph >> 32));
    s.v = __uint_as_float((uint32_t)vv);
  }
}

// ---------------------------------------------------------------------------
// Wavefront helpers

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t read_lane_u64(uint64_t x, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// 128-bit accumulation with two 64-bit atomics: the carry of the low word is
// known exactly from the value the atomic returns.
__device__ __forceinline__ void atomic_add_u128(unsigned long long* lo,
                                                unsigned long long* hi,
                                                unsigned long long add_lo,
                                                unsigned long long add_hi) {
  const unsigned long long old = atomicAdd(lo, add_lo);
  const unsigned long long carry = (old + add_lo < old) ? 1ull : 0ull;
  if (add_hi + carry) atomicAdd(hi, add_hi + carry);
}

// ---------------------------------------------------------------------------
// LDS result tables

struct LdsTables {
  uint32_t h_key[kHistSlots];
  uint32_t h_cnt[kHistSlots];
  uint32_t m_key[kMomSlots];
  unsigned long long m_val[kMomSlots][6];  // esc, cens, over, sum_k, k2 lo, hi
};

// Table slot of a key, (set << 12 | bin) or set: shifts and XORs only, so no
// multiplier constant is held in a scalar register for the whole kernel
// (the integrator's resident-wave count depends on those registers).
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  return x ^ (x >> 10) ^ (x >> 20);
}

// Per-set output description needed when a replica finishes.
struct SetOut {
  int64_t* out_steps;
  int64_t k_hist;
  double hist_scale;
  uint64_t hist_off;
  uint32_t n_bins;
};

__device__ __forceinline__ SetOut set_out(const SetDev& s) {
  return SetOut{s.out_steps, s.k_hist, s.hist_scale, s.hist_off, s.n_bins};
}

__device__ __forceinline__ uint32_t hist_bin(int64_t k, const SetOut& so) {
  return hist_bin_of(k, so.n_bins, so.k_hist, so.hist_scale);
}

__device__ void hist_add(LdsTables& t, const SliceArgs& a, uint32_t key,
                         uint32_t count, uint64_t global_index) {
  uint32_t h = hash32(key) & (kHistSlots - 1);
#pragma unroll 1
  for (int probe = 0; probe < kProbes; ++probe) {
    const uint32_t prev = atomicCAS(&t.h_key[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&t.h_cnt[h], count);
      return;
    }
    h = (h + 1) & (kHistSlots - 1);
  }
  atomicAdd(&a.hist[global_index], (unsigned long long)count);
}

__device__ void mom_add(LdsTables& t, const SliceArgs& a, uint32_t set,
                        int64_t k, bool overflow) {
  const unsigned long long esc = k > 0 ? 1ull : 0ull;
  const unsigned long long cens = 1ull - esc;
  const unsigned long long over = overflow ? 1ull : 0ull;
  const unsigned long long kk = k > 0 ? (unsigned long long)k : 0ull;
  const unsigned long long k2lo = kk * kk;
  const unsigned long long k2hi = __umul64hi(kk, kk);
  uint32_t h = hash32(set) & (kMomSlots - 1);
#pragma unroll 1
  for (int probe = 0; probe < kMomSlots; ++probe) {
    const uint32_t prev = atomicCAS(&t.m_key[h], kEmpty, set);
    if (prev == kEmpty || prev == set) {
      unsigned long long* v = t.m_val[h];
      if (esc) atomicAdd(&v[0], 1ull);
      if (cens) atomicAdd(&v[1], 1ull);
      if (over) atomicAdd(&v[2], 1ull);
      if (kk) {
        atomicAdd(&v[3], kk);
        atomic_add_u128(&v[4], &v[5], k2lo, k2hi);
      }
      return;
    }
    h = (h + 1) & (kMomSlots - 1);
  }
  MomDev* m = &a.mom[set];
  if (esc) atomicAdd(&m->n_esc, 1ull);
  if (cens) atomicAdd(&m->n_cens, 1ull);
  if (over) atomicAdd(&m->n_over, 1ull);
  if (kk) {
    atomicAdd(&m->sum_k, kk);
    atomic_add_u128(&m->sum_k2_lo, &m->sum_k2_hi, k2lo, k2hi);
  }
  atomicAdd(&a.ctr->done, 1ull);
}

// Record finished replicas of one slot across the wavefront.  `fin` lanes
// have finished with step k (k = -1: censored).
__device__ void record_finished(LdsTables& t, const SliceArgs& a, bool fin,
                                uint32_t set, uint64_t idx, int64_t k) {
  SetOut so{nullptr, 1, 1.0, 0, 1};
  uint32_t key = kEmpty;
  bool in_hist = false;
  if (fin) {
    so = set_out(a.sets[set]);
    if (so.out_steps) so.out_steps[idx] = k;
    if (k > 0 && k <= so.k_hist) {
      const uint32_t bin = hist_bin(k, so);
      key = (set << kBinBits) | bin;
      in_hist = true;
    }
    mom_add(t, a, set, k, k > so.k_hist);
  }
  // Wavefront merge: one LDS add per distinct (set, bin) among the lanes.
  uint64_t pending = __ballot(in_hist);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t lkey = __builtin_amdgcn_readlane((int)key, leader);
    const uint64_t same = __ballot(in_hist && key == lkey);
    if (lane_id() == (uint32_t)leader) {
      const uint32_t bin = key & ((1u << kBinBits) - 1);
      hist_add(t, a, key, (uint32_t)__popcll(same), so.hist_off + bin);
    }
    pending &= ~same;
  }
}

// ---------------------------------------------------------------------------
// Drawing replicas from the work queue.

// Grants up to `want` consecutive flat indices to the wavefront; returns the
// first in *base and the number granted.  Plans: plain atomicAdd (indices at
// or past `total` are simply empty).  Server: the cursor never passes
// `total`, so work appended later is not skipped.
__device__ __forceinline__ uint32_t draw(const SliceArgs& a, uint32_t want,
                                         unsigned long long* base) {
  if (!a.clamp) {
    const unsigned long long b = atomicAdd(&a.ctr->cursor, (unsigned long long)want);
    *base = b;
    if (b >= a.total) return 0;
    const unsigned long long avail = a.total - b;
    return avail < want ? (uint32_t)avail : want;
  }
  unsigned long long old = atomicAdd(&a.ctr->cursor, 0ull);
  for (;;) {
    const unsigned long long avail = old < a.total ? a.total - old : 0ull;
    const uint32_t take = avail < want ? (uint32_t)avail : want;
    if (take == 0) {
      *base = old;
      return 0;
    }
    const unsigned long long prev = atomicCAS(&a.ctr->cursor, old, old + take);
    if (prev == old) {
      *base = old;
      return take;
    }
    old = prev;
  }
}

// Flat index -> (set, replica).  False for padding inside a chunk.
__device__ __forceinline__ bool map_flat(const SliceArgs& a, uint64_t flat,
                                         uint32_t* set, uint64_t* idx) {
  if (a.chunks == nullptr) {
    *set = 0;
    *idx = flat;
    return true;
  }
  const Chunk ch = a.chunks[(flat / kChunk) & a.chunk_mask];
  const uint32_t off = (uint32_t)(flat % kChunk);
  *set = ch.set;
  *idx = ch.first + off;
  return off < ch.count;
}

// ---------------------------------------------------------------------------
// The integrator launch.

// Smallest value of x over the wavefront (rare paths only).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, off));
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// Blocks the active lanes of a slot can run before one of them reaches its
// last allowed block: min over active lanes of jmax - j (saturated).
template <bool FP64>
__device__ __forceinline__ uint32_t blocks_to_cap(const Slot<FP64>& sl, uint64_t jmax,
                                                  bool active) {
  uint32_t left = 0xFFFFFFFFu;
  if (active) {
    const uint64_t d = jmax > sl.j ? jmax - sl.j : 0ull;
    left = d > 0x7FFFFFFFull ? 0x7FFFFFFFu : (uint32_t)d;
  }
  return wave_min_u32(left);
}

// The 4 words of a slot's next block: Philox keyed by (block, replica) with
// the set's seed in scalar registers, or the next 4 outputs of the replica's
// MT19937 (active lanes only: a free slot's state is re-seeded when it takes
// a replica).
template <bool MT, bool FP64>
// (`pf`: the generator's parts for the slot's fixed counter words 1-3, for
// blocks whose low block word does not wrap; null: the full generator.)
__device__ __forceinline__ Words block_words(const SliceArgs& a, uint64_t n_slots,
                                             uint64_t slot, bool active, MtCarry& mc,
                                             const Slot<FP64>& sl, uint32_t k0,
                                             uint32_t k1, const PhiloxFixed* pf = nullptr) {
  if constexpr (MT) {
    Words w{0u, 0u, 0u, 0u};
    if (active) w = mt_block(a.st_mt, n_slots, slot, mc);
    return w;
  } else {
    if (pf) return philox4x32_10_fixed((uint32_t)sl.j, *pf, k0, k1);
    return philox4x32_10_uniform_key((uint32_t)sl.j, (uint32_t)(sl.j >> 32),
                                     (uint32_t)sl.idx, (uint32_t)(sl.idx >> 32), k0, k1);
  }
}

// Block index of the last allowed step of the slot's replica.
template <bool MULTI, bool FP64>
__device__ __forceinline__ uint64_t slot_jmax(const SliceArgs& a, const Slot<FP64>& sl,
                                              bool active, uint64_t jmax_one) {
  if constexpr (MULTI) {
    return active ? a.sets[sl.set].jmax : 0ull;
  } else {
    return jmax_one;
  }
}

// FP64: the 4 steps of a block for NR slots (r0 ... r0 + NR - 1) that share
// the constants P.  Where step q ends above the threshold, bit q of
// esc_bits[r] is set (PASS: the lanes of one pass of a multi-set block), or
// the wavefront masks esc[r][q] are formed directly.
template <int MODEL, int NR, bool MT, bool PASS>
__device__ __forceinline__ void block_f64(const SliceArgs& a, uint64_t n_slots,
                                          uint64_t lane_g, uint64_t lane_bit, int r0,
                                          const uint64_t* amask, MtCarry* mc,
                                          Slot<true>* s, const SetPar<true>& P,
                                          uint32_t* esc_bits, uint64_t (*esc)[4]) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    Slot<true>& sl = s[r];
    const Words w = block_words<MT>(a, n_slots, (uint64_t)(r0 + r) * a.n_lanes + lane_g,
                                    (amask[r] & lane_bit) != 0, mc[r], sl, P.k0, P.k1);
    double z[4];
    normals_f64(w, z);
    uint32_t bits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double kd = sl.kd + (double)q;
      if constexpr (MODEL == kUnderExplicit) {
        step_f64_under(P.p, kd, z[q], sl.phi, sl.v);
      } else if constexpr (MODEL == kUnderSemiImplicit) {
        step_f64_under_si(P.p, kd, z[q], sl.phi, sl.v);
      } else {
        step_f64_over(P.p, kd, z[q], sl.phi);
      }
      if constexpr (PASS) {
        bits |= (sl.phi > P.p.th) ? (1u << q) : 0u;
      } else {
        esc[r][q] = __ballot(sl.phi > P.p.th);
      }
    }
    if constexpr (PASS) esc_bits[r] = bits;
  }
}

// FP32C: the 4 steps of a block for NR slots sharing the constants P (gA:
// P.p.gA in a vector register).  Records the phase after each step for the
// threshold test that runs afterwards: ph_q[q] for q = 1..3 is the FP32
// phase x_q the next step sees, ph_q[4] the leading word of the new pair,
// whose error term is the slot's e (ph_q[0]: the block's start).
template <int MODEL, int NR, bool MT>
__device__ __forceinline__ void block_f32(const SliceArgs& a, uint64_t n_slots,
                                          uint64_t lane_g, uint64_t lane_bit, int r0,
                                          const uint64_t* amask, MtCarry* mc,
                                          Slot<false>* s, const SetPar<false>& P, double gA,
                                          float (*ph_q)[5], const PhiloxFixed* pf = nullptr) {
  const ParF32& p = P.p;
  // generator and normals of every slot first, then the 4 steps with the
  // slots interleaved (independent chains for the scheduler)
  BoxMullerF32 bm[NR];
  BlockG gk[NR];
  float zs[NR][2];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    Slot<false>& sl = s[r];
    // the bias terms first: independent of the generator, they fill its
    // dependency chain
    gk[r] = block_g4(p, sl.kd, gA);
    const Words w = block_words<MT>(a, n_slots, (uint64_t)(r0 + r) * a.n_lanes + lane_g,
                                    (amask[r] & lane_bit) != 0, mc[r], sl, P.k0, P.k1,
                                    pf ? pf + r : nullptr);
    bm[r] = box_muller_f32(w);
    // all four bias terms exist before the first step, so every step can
    // accumulate into its own (the first otherwise still feeds the rest)
    asm volatile("" : "+v"(gk[r].g[0]), "+v"(gk[r].g[1]), "+v"(gk[r].g[2]),
                 "+v"(gk[r].g[3]));
    zs[r][0] = p.sig * bm[r].radius[0];
    zs[r][1] = p.sig * bm[r].radius[1];
  }
  // the running sums start at the error terms, which they consume
  float d[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) d[r] = s[r].e;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      Slot<false>& sl = s[r];
      const float trig = (q & 1) ? bm[r].s[q >> 1] : bm[r].c[q >> 1];
      // the phase after step q: the block's start plus the running sum
      const float x = q == 0 ? sl.phi : sl.phi + d[r];
      ph_q[r][q] = x;
      if constexpr (MODEL == kUnderExplicit) {
        step_f32_under(p, gk[r].g[q], zs[r][q >> 1], trig, x, d[r], sl.v);
      } else if constexpr (MODEL == kUnderSemiImplicit) {
        step_f32_under_si(p, gk[r].g[q], zs[r][q >> 1], trig, x, d[r], sl.v);
      } else {
        step_f32_over(p, gk[r].g[q], zs[r][q >> 1], trig, x, d[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    fold_advance(d[r], s[r].phi, s[r].e);
    ph_q[r][4] = s[r].phi;
  }
}

// FP32C phase after step q of a block (q = 0..3) above the FP64 threshold:
// the FP32 phase itself after the first three, the compensated pair after
// the last (compared exactly in FP64 in both cases).
__device__ __forceinline__ bool above_after_step(const float (&ph_q)[5], float e, int q,
                                                 double th_rev) {
  return q == 3 ? above_f64(ph_q[4], e, th_rev) : (double)ph_q[q + 1] > th_rev;
}

// FP32C threshold test of one slot's block: one compare on the largest phase,
// and the exact FP64 test of each step only where an active lane came near
// the threshold (a finished lane keeps its last phase until it takes a new
// replica).
__device__ __forceinline__ void threshold_f32(const float (&ph_q)[5], float e,
                                              float th_near_rev, double th_rev,
                                              uint64_t amask, uint64_t (&esc)[4]) {
  esc[0] = esc[1] = esc[2] = esc[3] = 0ull;
  const float top = fmaxf(fmaxf(ph_q[1], ph_q[2]), fmaxf(ph_q[3], ph_q[4]));
  if (__ballot(top > th_near_rev) & amask) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      esc[q] = __ballot(ph_q[q + 1] > th_near_rev && above_after_step(ph_q, e, q, th_rev));
  }
}

// The same test for the lanes of one pass of a multi-set block: bit q of the
// result is set where step q ends above the threshold.
__device__ __forceinline__ uint32_t threshold_bits_f32(const float (&ph_q)[5], float e,
                                                       float th_near_rev, double th_rev) {
  uint32_t bits = 0;
  const float top = fmaxf(fmaxf(ph_q[1], ph_q[2]), fmaxf(ph_q[3], ph_q[4]));
  if (__ballot(top > th_near_rev)) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (ph_q[q + 1] > th_near_rev && above_after_step(ph_q, e, q, th_rev)) bits |= 1u << q;
  }
  return bits;
}

// End of a block for one slot: record the lanes whose replica crossed the
// threshold in one of the 4 steps (esc) or reached its step cap, free their
// slots, advance the block.  LANE_SET: the cap and step limit come from each
// lane's set; otherwise from set set_u, shared by all lanes (read from the
// table when needed, so they hold no registers through the block loop).
template <bool LANE_SET, bool FP64>
__device__ __forceinline__ void finish_slot(LdsTables& tab, const SliceArgs& a,
                                            Slot<FP64>& sl, uint64_t& amask, uint32_t& safe,
                                            const uint64_t (&esc)[4], uint64_t lane_bit,
                                            uint32_t set_u) {
  // The set's constants: set set_u, or for kInactive the set of the first
  // active lane (all active lanes share it).  Looked up only on the paths
  // that read them -- a step-cap check, a finished replica -- and always
  // first while amask still holds the block's lanes; the common block (no
  // finish, no cap check) does no lookup at all.
  uint32_t su_idx = set_u;
  auto su = [&]() -> const ConstSetDev& {
    if (!LANE_SET && su_idx == kInactive)
      su_idx = amask ? (uint32_t)__builtin_amdgcn_readlane(
                           (int)sl.set, __ffsll((unsigned long long)amask) - 1)
                     : 0u;
    return ((const ConstSetDev*)a.sets)[su_idx];
  };
  const uint64_t crossed = (esc[0] | esc[1] | esc[2] | esc[3]) & amask;
  const bool check_cap = safe == 0;
  uint64_t last = 0ull;
  if (check_cap) {
    const uint64_t jm = LANE_SET ? slot_jmax<true>(a, sl, (amask & lane_bit) != 0, 0ull)
                                 : su().jmax;
    last = __ballot(sl.j >= jm) & amask;
  }
  if (crossed | last) {
    const ConstSetDev* sp = LANE_SET ? nullptr : &su();
    bool fin = false;
    int64_t k = -1;
    if ((crossed | last) & lane_bit) {
      int q1 = 0;
      if (esc[0] & lane_bit) q1 = 1;
      else if (esc[1] & lane_bit) q1 = 2;
      else if (esc[2] & lane_bit) q1 = 3;
      else if (esc[3] & lane_bit) q1 = 4;
      const int64_t kesc = q1 ? (int64_t)(4 * sl.j) + q1 : 0;
      const int64_t max_steps = LANE_SET ? a.sets[sl.set].max_steps : sp->max_steps;
      if (q1 && kesc <= max_steps) {
        fin = true;
        k = kesc;
      } else if (sl.j >= (LANE_SET ? slot_jmax<true>(a, sl, true, 0ull) : sp->jmax)) {
        fin = true;
        k = -1;
      }
    }
    record_finished(tab, a, fin, sl.set, sl.idx, k);
    if (fin) sl.set = kInactive;
    amask &= ~__ballot(fin);
  }
  sl.j += 1;
  sl.kd += 4.0;
  if (check_cap) {
    const bool act = (amask & lane_bit) != 0;
    safe = blocks_to_cap(sl, LANE_SET ? slot_jmax<true>(a, sl, act, 0ull) : su().jmax, act);
  } else {
    --safe;
  }
}

// A multi-set wavefront integrates a block in passes, one per distinct set
// among the active lanes of a slot, each with that set's constants in scalar
// registers (the Philox key among them).  Lanes are grouped by set between
// launches, so nearly every block takes one pass; the passes beyond the first
// are counted for the host.
template <bool FP64, int MODEL, int R, bool MULTI, bool MT>
__device__ __forceinline__ void slice_body(const SliceArgs& a) {
  static_assert(!MT || (R == 1 && !MULTI), "MT19937 mode: one set, one slot per lane");
  __shared__ LdsTables tab;
  for (int i = threadIdx.x; i < kHistSlots; i += kBlockThreads) {
    tab.h_key[i] = kEmpty;
    tab.h_cnt[i] = 0;
  }
  for (int i = threadIdx.x; i < kMomSlots; i += kBlockThreads) {
    tab.m_key[i] = kEmpty;
#pragma unroll
    for (int f = 0; f < 6; ++f) tab.m_val[i][f] = 0ull;
  }
  __syncthreads();

  const uint64_t lane_g = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  const uint32_t lane = lane_id();
  const uint64_t lane_bit = 1ull << lane;

  // Constants of the set (of a single-set plan); gA also in one vector copy,
  // so the per-block FP64 fma reads a single scalar pair.  Multi-set
  // wavefronts load the constants of their lanes' set where they use them.
  SetPar<FP64> P{};
  double gA = 0.0;
  if constexpr (!MULTI) {
    P = load_setpar<FP64>(a.sets, 0);
    if constexpr (!FP64) {
      gA = P.p.gA;
      asm volatile("" : "+v"(gA));
    }
  }
  const uint64_t jmax_one = MULTI ? 0ull : ((ConstSetDev*)a.sets)[0].jmax;

  Slot<FP64> s[R];
  // activity of each slot as a wavefront mask, and the number of blocks all
  // its active lanes can run before one reaches its step cap
  uint64_t amask[R];
  uint32_t safe[R];
  MtCarry mc[R];
  const uint64_t n_slots = a.n_lanes * (uint64_t)R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    restore_slot(a, (uint64_t)r * a.n_lanes + lane_g, s[r]);
    const bool act = s[r].set != kInactive;
    if constexpr (MT) {
      const uint4 z4 = make_uint4(0, 0, 0, 0);
      mc[r] = MtCarry{z4, z4, z4, z4, 0u};
      if (act)
        mc[r] = mt_load(a.st_mt, n_slots, (uint64_t)r * a.n_lanes + lane_g,
                        (uint32_t)(s[r].j % kMtGroups));
    }
    amask[r] = __ballot(act);
    safe[r] = blocks_to_cap(s[r], slot_jmax<MULTI>(a, s[r], act, jmax_one), act);
  }

  bool starved = false;
  uint32_t blocks_run = 0;
  // (counted in a vector register: the scalar ones set the resident waves)
  uint32_t extra_passes = 0;
  asm volatile("" : "+v"(extra_passes));
  for (int blk = 0; blk < a.blocks; ++blk) {
    // ---- refill free slots
    if (a.refill && !starved) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint64_t need = ~amask[r];
        if (need && (!MULTI || !a.whole_waves || need == ~0ull)) {
          const uint32_t want = (uint32_t)__popcll(need);
          const int leader = __ffsll((unsigned long long)need) - 1;
          unsigned long long base = 0;
          uint32_t got = 0;
          if (lane == (uint32_t)leader) got = draw(a, want, &base);
          got = __builtin_amdgcn_readlane((int)got, leader);
          base = read_lane_u64(base, leader);
          if (got < want) starved = true;
          bool assigned = false;
          if (need & lane_bit) {
            const uint32_t rk = rank_in(need);
            uint32_t set;
            uint64_t idx;
            if (rk < got && map_flat(a, base + rk, &set, &idx)) {
              const SetDev& sd = a.sets[set];
              start_replica(s[r], set, idx, sd);
              if constexpr (MT) {
                const uint64_t slot = (uint64_t)r * a.n_lanes + lane_g;
                mt_seed_slot(a.st_mt, n_slots, slot, mt_replica_seed(sd.seed, idx));
                mc[r] = mt_load(a.st_mt, n_slots, slot, 0u);
              }
              assigned = true;
            }
          }
          const uint64_t newly = __ballot(assigned);
          if (newly) {
            amask[r] |= newly;
            const bool act = (amask[r] & lane_bit) != 0;
            safe[r] = blocks_to_cap(s[r], slot_jmax<MULTI>(a, s[r], act, jmax_one), act);
          }
        }
      }
    }
    uint64_t any = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) any |= amask[r];
    if (any == 0) break;
    ++blocks_run;

    if constexpr (!MULTI && R == 1 && !MT && !FP64) {
      // Every lane busy: run blocks without the refill test until one of
      // them finishes (its slot refills above in the next block) or the
      // launch ends.  (FP32C only: in the FP64 kernel the second copy of
      // the block costs more spilled scalar registers than the test.)  The
      // loop keeps each lane's replica, so the generator's counter words
      // 1-3 stay fixed unless a low block word wraps before the launch
      // ends (a replica past 2^32 blocks): where none can, their part of
      // the generator is formed once for the loop.
      const uint32_t left = (uint32_t)(a.blocks - blk);
      if (amask[0] == ~0ull && __ballot((uint32_t)s[0].j > 0xFFFFFFFFu - (left - 1u)) == 0) {
        const PhiloxFixed pf = philox_fixed_part((uint32_t)(s[0].j >> 32), (uint32_t)s[0].idx,
                                                 (uint32_t)(s[0].idx >> 32), P.k0, P.k1);
        for (;;) {
          uint64_t e1[1][4];
          float ph_q[1][5];
          block_f32<MODEL, 1, MT>(a, n_slots, lane_g, lane_bit, 0, amask, mc, s, P, gA, ph_q,
                                  &pf);
          threshold_f32(ph_q[0], s[0].e, P.p.th_near_rev, P.p.th_rev, amask[0], e1[0]);
          finish_slot<false>(tab, a, s[0], amask[0], safe[0], e1[0], lane_bit, 0u);
          if (amask[0] != ~0ull || blk + 1 >= a.blocks) break;
          ++blk;
          ++blocks_run;
        }
        continue;
      }
    }

    if constexpr (MULTI && R == 1) {
      // Wavefronts that refill only when free in every lane: while all active
      // lanes hold one set, run blocks with that set's constants fixed (the
      // single-set loop) until the wavefront is empty or the launch ends.
      if (a.whole_waves) {
        const uint32_t s_first = (uint32_t)__builtin_amdgcn_readlane(
            (int)s[0].set, __ffsll((unsigned long long)amask[0]) - 1);
        // (FP32C with Philox: also no active lane's low block word may wrap
        // before the launch ends, so that the generator's fixed counter
        // words hold for the loop, as in the single-set busy loop)
        constexpr bool kFixed = !FP64 && !MT;
        const uint32_t left = (uint32_t)(a.blocks - blk);
        if ((__ballot(s[0].set != s_first) & amask[0]) == 0 &&
            (!kFixed ||
             (__ballot((uint32_t)s[0].j > 0xFFFFFFFFu - (left - 1u)) & amask[0]) == 0)) {
          const SetPar<FP64> Q = load_setpar<FP64>(a.sets, s_first);
          double gQ = 0.0;
          PhiloxFixed pf{};
          if constexpr (!FP64) {
            gQ = Q.p.gA;
            asm volatile("" : "+v"(gQ));
          }
          if constexpr (kFixed)
            pf = philox_fixed_part((uint32_t)(s[0].j >> 32), (uint32_t)s[0].idx,
                                   (uint32_t)(s[0].idx >> 32), Q.k0, Q.k1);
          for (;;) {
            uint64_t e1[1][4];
            if constexpr (FP64) {
              block_f64<MODEL, 1, MT, false>(a, n_slots, lane_g, lane_bit, 0, amask, mc, s, Q,
                                             nullptr, e1);
            } else {
              float ph_q[1][5];
              block_f32<MODEL, 1, MT>(a, n_slots, lane_g, lane_bit, 0, amask, mc, s, Q, gQ,
                                      ph_q, kFixed ? &pf : nullptr);
              threshold_f32(ph_q[0], s[0].e, Q.p.th_near_rev, Q.p.th_rev, amask[0], e1[0]);
            }
            finish_slot<false>(tab, a, s[0], amask[0], safe[0], e1[0], lane_bit, kInactive);
            if (amask[0] == 0 || blk + 1 >= a.blocks) break;
            ++blk;
            ++blocks_run;
          }
          continue;
        }
      }
    }

    // ---- 4 Euler steps per slot, then the threshold test
    uint64_t esc[R][4];
    if constexpr (!MULTI) {
      if constexpr (FP64) {
        block_f64<MODEL, R, MT, false>(a, n_slots, lane_g, lane_bit, 0, amask, mc, s, P,
                                       nullptr, esc);
      } else {
        float ph_q[R][5];
        block_f32<MODEL, R, MT>(a, n_slots, lane_g, lane_bit, 0, amask, mc, s, P, gA, ph_q);
#pragma unroll
        for (int r = 0; r < R; ++r)
          threshold_f32(ph_q[r], s[r].e, P.p.th_near_rev, P.p.th_rev, amask[r], esc[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // the set of the first active lane; one pass at full width when every
        // active lane has it, else one pass per set
        const uint64_t todo0 = amask[r];
        const uint32_t s_first =
            todo0 ? (uint32_t)__builtin_amdgcn_readlane(
                        (int)s[r].set, __ffsll((unsigned long long)todo0) - 1)
                  : 0u;
        // (one-slot kernels reach this point with mixed wavefronts, or
        // without whole-wavefront refill: passes only, one body less)
        if (R > 1 && (__ballot(s[r].set != s_first) & todo0) == 0) {
          const SetPar<FP64> Q = load_setpar<FP64>(a.sets, s_first);
          if constexpr (FP64) {
            block_f64<MODEL, 1, MT, false>(a, n_slots, lane_g, lane_bit, r, &amask[r], &mc[r],
                                           &s[r], Q, nullptr, &esc[r]);
          } else {
            double gQ = Q.p.gA;
            asm volatile("" : "+v"(gQ));
            float ph_q[5];
            block_f32<MODEL, 1, MT>(a, n_slots, lane_g, lane_bit, r, &amask[r], &mc[r], &s[r],
                                    Q, gQ, &ph_q);
            threshold_f32(ph_q, s[r].e, Q.p.th_near_rev, Q.p.th_rev, amask[r], esc[r]);
          }
        } else {
          // a lane is in the pass of set s0 exactly when its set is s0 (a
          // free lane's set is kInactive); each pass tests its own lanes
          // against its set's threshold and leaves per-lane escape bits
          uint32_t bits = 0;
          for (uint64_t todo = todo0; todo;) {
            const uint32_t s0 = (uint32_t)__builtin_amdgcn_readlane(
                (int)s[r].set, __ffsll((unsigned long long)todo) - 1);
            const bool mine = s[r].set == s0;
            todo &= ~__ballot(mine);
            const SetPar<FP64> Q = load_setpar<FP64>(a.sets, s0);
            if (mine) {
              if constexpr (FP64) {
                block_f64<MODEL, 1, MT, true>(a, n_slots, lane_g, lane_bit, r, &amask[r],
                                              &mc[r], &s[r], Q, &bits, nullptr);
              } else {
                double gQ = Q.p.gA;
                asm volatile("" : "+v"(gQ));
                float ph_q[5];
                block_f32<MODEL, 1, MT>(a, n_slots, lane_g, lane_bit, r, &amask[r], &mc[r],
                                        &s[r], Q, gQ, &ph_q);
                bits = threshold_bits_f32(ph_q, s[r].e, Q.p.th_near_rev, Q.p.th_rev);
              }
            }
            if (todo) ++extra_passes;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) esc[r][q] = __ballot((bits >> q) & 1u);
        }
      }
    }

    // ---- escapes, censoring, next block
#pragma unroll
    for (int r = 0; r < R; ++r)
      finish_slot<MULTI>(tab, a, s[r], amask[r], safe[r], esc[r], lane_bit, 0u);
  }

  // ---- leave state resident, count issued lane-steps
#pragma unroll
  for (int r = 0; r < R; ++r) store_slot(a, (uint64_t)r * a.n_lanes + lane_g, s[r]);
  if (lane == 0 && blocks_run)
    atomicAdd(&a.ctr->lane_steps,
              (unsigned long long)blocks_run * (unsigned long long)(kWave * R * 4));
  if (MULTI && lane == 0 && extra_passes)
    atomicAdd(&a.ctr->extra_passes, (unsigned long long)extra_passes);

  // ---- one global pass over the workgroup's LDS tables
  __syncthreads();
  for (int i = threadIdx.x; i < kHistSlots; i += kBlockThreads) {
    const uint32_t key = tab.h_key[i];
    if (key != kEmpty && tab.h_cnt[i]) {
      const uint32_t set = key >> kBinBits;
      const uint32_t bin = key & ((1u << kBinBits) - 1);
      const uint64_t off = a.sets[set].hist_off;
      atomicAdd(&a.hist[off + bin], (unsigned long long)tab.h_cnt[i]);
    }
  }
  for (int i = threadIdx.x; i < kMomSlots; i += kBlockThreads) {
    const uint32_t set = tab.m_key[i];
    if (set == kEmpty) continue;
    const unsigned long long* v = tab.m_val[i];
    MomDev* m = &a.mom[set];
    if (v[0]) atomicAdd(&m->n_esc, v[0]);
    if (v[1]) atomicAdd(&m->n_cens, v[1]);
    if (v[2]) atomicAdd(&m->n_over, v[2]);
    if (v[3]) atomicAdd(&m->sum_k, v[3]);
    if (v[4] | v[5]) atomic_add_u128(&m->sum_k2_lo, &m->sum_k2_hi, v[4], v[5]);
    if (v[0] + v[1]) atomicAdd(&a.ctr->done, v[0] + v[1]);
  }
}

// (The FP32C one-slot kernels, single- and multi-set, fit 8 waves per SIMD
// on their own: 50-58 VGPRs, 93-99 SGPRs, no spill.  Asking the compiler
// for 8 waves as well capped the multi-set kernel at 78 SGPRs and spilled
// 26 of them through VGPR lanes.)
template <bool FP64, int MODEL, int R, bool MULTI, bool MT>
__global__ __launch_bounds__(kBlockThreads) void slice_kernel(SliceArgs a) {
  slice_body<FP64, MODEL, R, MULTI, MT>(a);
}

// ---------------------------------------------------------------------------
// Start of a run: slot i takes flat replica i (if any); all others are free.

template <bool FP64>
__global__ __launch_bounds__(kBlockThreads) void init_kernel(SliceArgs a,
                                                             uint64_t n_slots,
                                                             uint64_t n_assign) {
  const uint64_t slot = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  if (slot >= n_slots) return;
  Slot<FP64> s;
  s.set = kInactive;
  s.idx = 0;
  s.j = 0;
  s.kd = 0.0;
  s.phi = 0;
  s.v = 0;
  s.e = 0.0f;
  uint32_t set;
  uint64_t idx;
  if (slot < n_assign && map_flat(a, slot, &set, &idx)) {
    start_replica(s, set, idx, a.sets[set]);
    if (a.st_mt)
      mt_seed_slot(a.st_mt, n_slots, slot, mt_replica_seed(a.sets[set].seed, idx));
  }
  store_slot(a, slot, s);
}

// ---------------------------------------------------------------------------
// Tail compaction: once no undrawn replica is left, the active slots' state
// moves to a dense prefix of another state buffer, so later launches need
// fewer workgroups and no wave runs mostly idle lanes.  Which slot runs a
// replica does not change its results.

// Wavefront-aggregated claim of consecutive positions for the flagged lanes.
__device__ __forceinline__ uint64_t claim_positions(unsigned long long* counter,
                                                    bool flag) {
  const uint64_t mask = __ballot(flag);
  if (mask == 0) return 0;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == (uint32_t)leader)
    base = atomicAdd(counter, (unsigned long long)__popcll(mask));
  base = read_lane_u64(base, leader);
  return base + rank_in(mask);
}

__global__ __launch_bounds__(kBlockThreads) void compact_count_kernel(SliceArgs a,
                                                                      uint64_t n_slots) {
  const uint64_t slot = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  const bool act = slot < n_slots && a.st_set[slot] != kInactive;
  (void)claim_positions(&a.ctr->compact, act);
}

// dst's set array must already mark every slot inactive.
__global__ __launch_bounds__(kBlockThreads) void compact_move_kernel(SliceArgs src,
                                                                     SliceArgs dst,
                                                                     uint64_t n_slots) {
  const uint64_t slot = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  const uint32_t set = slot < n_slots ? src.st_set[slot] : kInactive;
  const bool act = set != kInactive;
  const uint64_t pos = claim_positions(&src.ctr->compact, act);
  if (!act) return;
  dst.st_set[pos] = set;
  dst.st_idx[pos] = src.st_idx[slot];
  dst.st_j[pos] = src.st_j[slot];
  dst.st_phi[pos] = src.st_phi[slot];
  dst.st_v[pos] = src.st_v[slot];
}

// ---------------------------------------------------------------------------
// Grouping by set: the active slots' state moves to another state buffer in
// the order of their sets, so the lanes of a wavefront share a set and a
// multi-set block takes one pass.  Counting per set, an exclusive scan into
// first positions, then the move, which claims positions within its set.
// Each workgroup takes a contiguous tile of slots (after the first regroup
// they are in set order, so a tile holds few sets), sums per set in an LDS
// table and makes one global atomic per set it holds; sets beyond the
// table's capacity fall back to one atomic per wavefront.

// Wavefront-aggregated claim of the next position of counter[key] by each
// flagged lane: one atomic per distinct key among the lanes.
__device__ __forceinline__ uint64_t claim_by_key(unsigned long long* counter, uint32_t key,
                                                 bool flag) {
  const uint64_t lane_bit = 1ull << lane_id();
  uint64_t pending = __ballot(flag);
  uint64_t pos = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t lkey = __builtin_amdgcn_readlane((int)key, leader);
    const uint64_t same = __ballot(flag && key == lkey) & pending;
    unsigned long long base = 0;
    if (lane_id() == (uint32_t)leader)
      base = atomicAdd(&counter[lkey], (unsigned long long)__popcll(same));
    base = read_lane_u64(base, leader);
    if (same & lane_bit) pos = base + rank_in(same);
    pending &= ~same;
  }
  return pos;
}

constexpr int kGroupPerThread = 8;                               // slots per thread
constexpr int kGroupTile = kBlockThreads * kGroupPerThread;      // slots per workgroup
constexpr int kGroupTable = 128;                                 // LDS entries (sets)
constexpr uint32_t kNoEntry = 0xFFFFFFFFu;

struct GroupTable {
  uint32_t key[kGroupTable];
  uint32_t cnt[kGroupTable];
  unsigned long long base[kGroupTable];
};

__device__ __forceinline__ void group_table_init(GroupTable& t) {
  for (int i = threadIdx.x; i < kGroupTable; i += kBlockThreads) {
    t.key[i] = kEmpty;
    t.cnt[i] = 0;
  }
}

// Adds the wavefront's flagged lanes to the table, one LDS atomic per
// distinct set; returns this lane's entry (kNoEntry: table full, or unflagged).
__device__ __forceinline__ uint32_t group_table_add(GroupTable& t, uint32_t set, bool flag) {
  uint64_t pending = __ballot(flag);
  uint32_t entry = kNoEntry;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t lset = (uint32_t)__builtin_amdgcn_readlane((int)set, leader);
    const uint64_t same = __ballot(flag && set == lset) & pending;
    uint32_t e = kNoEntry;
    if (lane_id() == (uint32_t)leader) {
      uint32_t h = hash32(lset) & (kGroupTable - 1);
      for (int probe = 0; probe < kGroupTable; ++probe) {
        const uint32_t prev = atomicCAS(&t.key[h], kEmpty, lset);
        if (prev == kEmpty || prev == lset) {
          atomicAdd(&t.cnt[h], (uint32_t)__popcll(same));
          e = h;
          break;
        }
        h = (h + 1) & (kGroupTable - 1);
      }
    }
    e = (uint32_t)__builtin_amdgcn_readlane((int)e, leader);
    if (same & (1ull << lane_id())) entry = e;
    pending &= ~same;
  }
  return entry;
}

// counts[set] += active slots of the set (counts are zero before).
__global__ __launch_bounds__(kBlockThreads) void group_count_kernel(SliceArgs a,
                                                                    uint64_t n_slots,
                                                                    unsigned long long* counts) {
  __shared__ GroupTable t;
  group_table_init(t);
  __syncthreads();
  const uint64_t tile = (uint64_t)blockIdx.x * kGroupTile;
#pragma unroll
  for (int i = 0; i < kGroupPerThread; ++i) {
    const uint64_t slot = tile + (uint64_t)i * kBlockThreads + threadIdx.x;
    const uint32_t set = slot < n_slots ? a.st_set[slot] : kInactive;
    const bool act = set != kInactive;
    const uint32_t e = group_table_add(t, set, act);
    (void)claim_by_key(counts, set, act && e == kNoEntry);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kGroupTable; i += kBlockThreads)
    if (t.key[i] != kEmpty) atomicAdd(&counts[t.key[i]], (unsigned long long)t.cnt[i]);
}

// first[i] = exclusive prefix sum of counts rounded up to multiples of
// `align` (64: every set's slots start a wavefront, so none holds two sets),
// counts cleared for the next regroup, the total in ctr->compact.  One
// workgroup: each thread sums a contiguous range, a wavefront scan and an
// LDS pass combine the ranges.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void group_scan_kernel(unsigned long long* counts,
                                                                  unsigned long long* first,
                                                                  uint64_t n, uint32_t align,
                                                                  Counters* ctr) {
  __shared__ unsigned long long wave_sum[kScanThreads / kWave];
  const uint64_t per = (n + kScanThreads - 1) / kScanThreads;
  const uint64_t b = (uint64_t)threadIdx.x * per;
  const uint64_t e = b + per < n ? b + per : n;
  const unsigned long long m = align - 1;
  unsigned long long sum = 0;
  for (uint64_t i = b; i < e; ++i) sum += (counts[i] + m) & ~m;
  // inclusive scan of the thread sums within the wavefront
  const uint32_t lane = lane_id();
  unsigned long long incl = sum;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const unsigned long long up = ((unsigned long long)(uint32_t)__shfl_up((int)(uint32_t)(incl >> 32), off) << 32) |
                                  (uint32_t)__shfl_up((int)(uint32_t)incl, off);
    if (lane >= (uint32_t)off) incl += up;
  }
  const int wave = threadIdx.x / kWave;
  if (lane == kWave - 1) wave_sum[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
      const unsigned long long v = wave_sum[w];
      wave_sum[w] = run;
      run += v;
    }
    ctr->compact = run;
  }
  __syncthreads();
  unsigned long long run = wave_sum[wave] + incl - sum;
  for (uint64_t i = b; i < e; ++i) {
    const unsigned long long v = (counts[i] + m) & ~m;
    first[i] = run;
    counts[i] = 0;
    run += v;
  }
}

// Moves each active slot of the tile to the next position of its set
// (first[] from the scan): the tile's count per set reserves one range per
// set with a global atomic, the lanes take positions in it from LDS.  dst's
// set array must already mark every slot inactive.
__global__ __launch_bounds__(kBlockThreads) void group_move_kernel(SliceArgs src, SliceArgs dst,
                                                                   uint64_t n_slots,
                                                                   uint64_t n_dst_slots,
                                                                   unsigned long long* first) {
  __shared__ GroupTable t;
  group_table_init(t);
  __syncthreads();
  const uint64_t tile = (uint64_t)blockIdx.x * kGroupTile;
  uint32_t set[kGroupPerThread], entry[kGroupPerThread];
#pragma unroll
  for (int i = 0; i < kGroupPerThread; ++i) {
    const uint64_t slot = tile + (uint64_t)i * kBlockThreads + threadIdx.x;
    set[i] = slot < n_slots ? src.st_set[slot] : kInactive;
    entry[i] = group_table_add(t, set[i], set[i] != kInactive);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kGroupTable; i += kBlockThreads) {
    if (t.key[i] != kEmpty) {
      t.base[i] = atomicAdd(&first[t.key[i]], (unsigned long long)t.cnt[i]);
      t.cnt[i] = 0;
    }
  }
  __syncthreads();
  const uint64_t lane_bit = 1ull << lane_id();
#pragma unroll
  for (int i = 0; i < kGroupPerThread; ++i) {
    const uint64_t slot = tile + (uint64_t)i * kBlockThreads + threadIdx.x;
    const bool act = set[i] != kInactive;
    const bool in_table = act && entry[i] != kNoEntry;
    // positions from the tile's reservation, one LDS atomic per entry
    uint64_t pos = 0;
    uint64_t pending = __ballot(in_table);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t le = (uint32_t)__builtin_amdgcn_readlane((int)entry[i], leader);
      const uint64_t same = __ballot(in_table && entry[i] == le) & pending;
      uint32_t off = 0;
      if (lane_id() == (uint32_t)leader) off = atomicAdd(&t.cnt[le], (uint32_t)__popcll(same));
      off = (uint32_t)__builtin_amdgcn_readlane((int)off, leader);
      if (same & lane_bit) pos = t.base[le] + off + rank_in(same);
      pending &= ~same;
    }
    // sets the table could not hold: one global atomic per wavefront
    const uint64_t pos_g = claim_by_key(first, set[i], act && !in_table);
    if (act && !in_table) pos = pos_g;
    // positions stay below the aligned total, which fits the slots while
    // every wavefront holds one set; anything else is counted, not written
    if (act && pos >= n_dst_slots) atomicAdd(&src.ctr->overflow, 1ull);
    if (act && pos < n_dst_slots) {
      dst.st_set[pos] = set[i];
      dst.st_idx[pos] = src.st_idx[slot];
      dst.st_j[pos] = src.st_j[slot];
      dst.st_phi[pos] = src.st_phi[slot];
      dst.st_v[pos] = src.st_v[slot];
    }
  }
}

// After a move in set order (the sets' wavefront-aligned slots fill
// [0, ctr->compact)), the free slots past them take the next undrawn replicas
// in queue order.  The cursor stays a multiple of 64 (so does every draw of a
// whole wavefront), so each new wavefront holds one work-queue chunk: one set.
// (The cursor moves past them in copy_state_kernel, which runs next.)
template <bool FP64>
__global__ __launch_bounds__(kBlockThreads) void group_refill_kernel(SliceArgs a,
                                                                     uint64_t n_slots) {
  const uint64_t pos = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  const uint64_t active = a.ctr->compact;
  const uint64_t cursor = a.ctr->cursor;
  if (pos >= n_slots || pos < active || cursor >= a.total) return;
  const uint64_t flat = cursor + (pos - active);
  uint32_t set;
  uint64_t idx;
  if (flat >= a.total || !map_flat(a, flat, &set, &idx)) return;
  Slot<FP64> s;
  start_replica(s, set, idx, a.sets[set]);
  store_slot(a, pos, s);
}

// Lane state of n_slots slots from src to dst; with `advance`, also the
// cursor past the replicas the refill took (never past `total`).
__global__ __launch_bounds__(kBlockThreads) void copy_state_kernel(SliceArgs src, SliceArgs dst,
                                                                   uint64_t n_slots,
                                                                   int advance) {
  const uint64_t slot = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  if (advance && slot == 0) {
    Counters* ctr = src.ctr;
    const unsigned long long active = ctr->compact;
    const unsigned long long cursor = ctr->cursor;
    if (cursor < src.total) {
      const unsigned long long free = active < n_slots ? n_slots - active : 0ull;
      const unsigned long long left = src.total - cursor;
      ctr->cursor = cursor + (free < left ? free : left);
    }
  }
  if (slot >= n_slots) return;
  dst.st_set[slot] = src.st_set[slot];
  dst.st_idx[slot] = src.st_idx[slot];
  dst.st_j[slot] = src.st_j[slot];
  dst.st_phi[slot] = src.st_phi[slot];
  dst.st_v[slot] = src.st_v[slot];
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t value) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void fill_u64_kernel(unsigned long long* p, uint64_t n,
                                unsigned long long value) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// ---------------------------------------------------------------------------
// Diagnostics: the same device functions as the integrator.

__global__ void rng_words_kernel(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                                 uint64_t block0, uint64_t n_blk, uint32_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rep * n_blk) return;
  const uint64_t r = i / n_blk, b = i % n_blk;
  const Words w = replica_words(seed, replica0 + r, block0 + b);
  out[4 * i + 0] = w.w0;
  out[4 * i + 1] = w.w1;
  out[4 * i + 2] = w.w2;
  out[4 * i + 3] = w.w3;
}

template <bool FP64>
__global__ void normals_kernel(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                               uint64_t block0, uint64_t n_blk, void* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rep * n_blk) return;
  const uint64_t r = i / n_blk, b = i % n_blk;
  const Words w = replica_words(seed, replica0 + r, block0 + b);
  if constexpr (FP64) {
    double z[4];
    normals_f64(w, z);
    for (int q = 0; q < 4; ++q) static_cast<double*>(out)[4 * i + q] = z[q];
  } else {
    float z[4];
    normals_f32(w, z);
    for (int q = 0; q < 4; ++q) static_cast<float*>(out)[4 * i + q] = z[q];
  }
}

// One lane per replica, state at st (n_rep slots).
__global__ void mt_words_kernel(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                                uint64_t block0, uint64_t n_blk, uint4* st,
                                uint32_t* out) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rep) return;
  mt_seed_slot(st, n_rep, r, mt_replica_seed(seed, replica0 + r));
  MtCarry mc = mt_load(st, n_rep, r, 0u);
  for (uint64_t b = 0; b < block0 + n_blk; ++b) {
    const Words w = mt_block(st, n_rep, r, mc);
    if (b < block0) continue;
    uint32_t* o = out + 4 * (r * n_blk + (b - block0));
    o[0] = w.w0;
    o[1] = w.w1;
    o[2] = w.w2;
    o[3] = w.w3;
  }
}

template <bool FP64, int MODEL>
__global__ void trajectory_kernel(SetDev sd, uint64_t replica, int64_t n_steps,
                                  double* out_phi, double* out_v, uint4* mt) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Slot<FP64> s;
  start_replica(s, 0, replica, sd);
  SetPar<FP64> P;
  if constexpr (FP64) {
    P.p = load_par_f64(sd);
  } else {
    P.p = load_par_f32(sd);
  }
  MtCarry mc{make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0),
             make_uint4(0, 0, 0, 0), 0u};
  if (mt) {
    mt_seed_slot(mt, 1, 0, mt_replica_seed(sd.seed, replica));
    mc = mt_load(mt, 1, 0, 0u);
  }
  for (int64_t k0 = 0; k0 < n_steps; k0 += 4) {
    const Words w = mt ? mt_block(mt, 1, 0, mc) : replica_words(sd.seed, replica, s.j);
    if constexpr (FP64) {
      double z[4];
      normals_f64(w, z);
      for (int q = 0; q < 4 && k0 + q < n_steps; ++q) {
        const double kd = s.kd + (double)q;
        if constexpr (MODEL == kUnderExplicit) {
          step_f64_under(P.p, kd, z[q], s.phi, s.v);
        } else if constexpr (MODEL == kUnderSemiImplicit) {
          step_f64_under_si(P.p, kd, z[q], s.phi, s.v);
        } else {
          step_f64_over(P.p, kd, z[q], s.phi);
        }
        out_phi[k0 + q] = s.phi;
        out_v[k0 + q] = s.v;
      }
    } else {
      const BoxMullerF32 bm = box_muller_f32(w);
      const BlockG gk = block_g4(P.p, s.kd, P.p.gA);
      float d = s.e;
      for (int q = 0; q < 4 && k0 + q < n_steps; ++q) {
        const float zs = P.p.sig * bm.radius[q >> 1];
        const float trig = (q & 1) ? bm.s[q >> 1] : bm.c[q >> 1];
        const float x = q == 0 ? s.phi : s.phi + d;
        if constexpr (MODEL == kUnderExplicit) {
          step_f32_under(P.p, gk.g[q], zs, trig, x, d, s.v);
        } else if constexpr (MODEL == kUnderSemiImplicit) {
          step_f32_under_si(P.p, gk.g[q], zs, trig, x, d, s.v);
        } else {
          step_f32_over(P.p, gk.g[q], zs, trig, x, d);
        }
        // the phase the integrator tests after this step
        if (q < 3) {
          out_phi[k0 + q] = 2.0 * kPi * (double)(s.phi + d);
        } else {
          fold_advance(d, s.phi, s.e);
          out_phi[k0 + q] = 2.0 * kPi * ((double)s.phi + (double)s.e);
        }
        out_v[k0 + q] = (double)s.v;
      }
    }
    s.j += 1;
    s.kd += 4.0;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers

// The slice kernel instance for (precision, kind, R, multi, MT).
template <bool FP64, int MODEL, int R>
static const void* slice_ptr_m(bool multi, bool mt) {
  if constexpr (R == 1) {
    if (mt) return multi ? nullptr : (const void*)&slice_kernel<FP64, MODEL, 1, false, true>;
  } else {
    if (mt) return nullptr;
  }
  return multi ? (const void*)&slice_kernel<FP64, MODEL, R, true, false>
               : (const void*)&slice_kernel<FP64, MODEL, R, false, false>;
}

template <bool FP64>
static const void* slice_ptr_k(int kind, int R, bool multi, bool mt) {
  switch (kind) {
    case kOver:
      return R == 2 ? slice_ptr_m<FP64, kOver, 2>(multi, mt)
                    : slice_ptr_m<FP64, kOver, 1>(multi, mt);
    case kUnderSemiImplicit:
      return R == 2 ? slice_ptr_m<FP64, kUnderSemiImplicit, 2>(multi, mt)
                    : slice_ptr_m<FP64, kUnderSemiImplicit, 1>(multi, mt);
    default:
      return R == 2 ? slice_ptr_m<FP64, kUnderExplicit, 2>(multi, mt)
                    : slice_ptr_m<FP64, kUnderExplicit, 1>(multi, mt);
  }
}

static const void* slice_ptr(bool fp64, int kind, int R, bool multi, bool mt) {
  if (R != 1 && R != 2) return nullptr;
  return fp64 ? slice_ptr_k<true>(kind, R, multi, mt) : slice_ptr_k<false>(kind, R, multi, mt);
}

hipError_t launch_slice(bool fp64, int kind, int R, bool multi,
                        const SliceArgs& a, uint32_t n_groups, hipStream_t st) {
  const void* f = slice_ptr(fp64, kind, R, multi, a.st_mt != nullptr);
  if (!f) return hipErrorInvalidValue;
  SliceArgs args = a;
  void* params[] = {&args};
  return hipLaunchKernel(f, dim3(n_groups), dim3(kBlockThreads), params, 0, st);
}

int slice_resident_groups(bool fp64, int kind, int R, bool multi, bool mt) {
  const void* f = slice_ptr(fp64, kind, R, multi, mt);
  int n = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlockThreads, 0) !=
                hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

hipError_t launch_init(bool fp64, const SliceArgs& a, uint64_t n_slots,
                       uint64_t n_assign, hipStream_t st) {
  const uint32_t groups = (uint32_t)((n_slots + kBlockThreads - 1) / kBlockThreads);
  if (groups == 0) return hipSuccess;
  if (fp64) {
    hipLaunchKernelGGL(init_kernel<true>, dim3(groups), dim3(kBlockThreads), 0, st,
                       a, n_slots, n_assign);
  } else {
    hipLaunchKernelGGL(init_kernel<false>, dim3(groups), dim3(kBlockThreads), 0, st,
                       a, n_slots, n_assign);
  }
  return hipGetLastError();
}

hipError_t launch_compact_count(const SliceArgs& a, uint64_t n_slots, hipStream_t st) {
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(compact_count_kernel,
                     dim3((uint32_t)((n_slots + kBlockThreads - 1) / kBlockThreads)),
                     dim3(kBlockThreads), 0, st, a, n_slots);
  return hipGetLastError();
}

hipError_t launch_compact_move(const SliceArgs& src, const SliceArgs& dst, uint64_t n_slots,
                               uint64_t n_dst_slots, hipStream_t st) {
  if (n_dst_slots > 0) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)((n_dst_slots + 255) / 256)), dim3(256),
                       0, st, dst.st_set, n_dst_slots, kInactive);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(compact_move_kernel,
                     dim3((uint32_t)((n_slots + kBlockThreads - 1) / kBlockThreads)),
                     dim3(kBlockThreads), 0, st, src, dst, n_slots);
  return hipGetLastError();
}

hipError_t launch_group_count(const SliceArgs& a, uint64_t n_slots, unsigned long long* counts,
                              unsigned long long* first, uint64_t n_sets, hipStream_t st) {
  if (n_sets == 0) return hipSuccess;
  if (n_slots > 0) {
    hipLaunchKernelGGL(group_count_kernel,
                       dim3((uint32_t)((n_slots + kGroupTile - 1) / kGroupTile)),
                       dim3(kBlockThreads), 0, st, a, n_slots, counts);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, counts, first, n_sets,
                     (uint32_t)kWave, a.ctr);
  return hipGetLastError();
}

hipError_t launch_group_move(const SliceArgs& src, const SliceArgs& dst, uint64_t n_slots,
                             uint64_t n_dst_slots, unsigned long long* first, hipStream_t st) {
  if (n_dst_slots > 0) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)((n_dst_slots + 255) / 256)), dim3(256),
                       0, st, dst.st_set, n_dst_slots, kInactive);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(group_move_kernel, dim3((uint32_t)((n_slots + kGroupTile - 1) / kGroupTile)),
                     dim3(kBlockThreads), 0, st, src, dst, n_slots, n_dst_slots, first);
  return hipGetLastError();
}

hipError_t launch_group_refill(bool fp64, const SliceArgs& a, uint64_t n_slots,
                               hipStream_t st) {
  if (n_slots == 0) return hipSuccess;
  const dim3 g((uint32_t)((n_slots + kBlockThreads - 1) / kBlockThreads));
  if (fp64) {
    hipLaunchKernelGGL(group_refill_kernel<true>, g, dim3(kBlockThreads), 0, st, a, n_slots);
  } else {
    hipLaunchKernelGGL(group_refill_kernel<false>, g, dim3(kBlockThreads), 0, st, a, n_slots);
  }
  return hipGetLastError();
}

hipError_t launch_copy_state(const SliceArgs& src, const SliceArgs& dst, uint64_t n_slots,
                             bool advance_cursor, hipStream_t st) {
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_state_kernel,
                     dim3((uint32_t)((n_slots + kBlockThreads - 1) / kBlockThreads)),
                     dim3(kBlockThreads), 0, st, src, dst, n_slots, advance_cursor ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n,
                           unsigned long long value, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint32_t groups = (uint32_t)((n + 255) / 256);
  hipLaunchKernelGGL(fill_u64_kernel, dim3(groups), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_rng_words(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                            uint64_t block0, uint64_t n_blk, uint32_t* out,
                            hipStream_t st) {
  const uint64_t n = n_rep * n_blk;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(rng_words_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256),
                     0, st, seed, replica0, n_rep, block0, n_blk, out);
  return hipGetLastError();
}

hipError_t launch_normals(bool fp64, uint64_t seed, uint64_t replica0,
                          uint64_t n_rep, uint64_t block0, uint64_t n_blk,
                          void* out, hipStream_t st) {
  const uint64_t n = n_rep * n_blk;
  if (n == 0) return hipSuccess;
  const dim3 g((uint32_t)((n + 255) / 256));
  if (fp64) {
    hipLaunchKernelGGL(normals_kernel<true>, g, dim3(256), 0, st, seed, replica0,
                       n_rep, block0, n_blk, out);
  } else {
    hipLaunchKernelGGL(normals_kernel<false>, g, dim3(256), 0, st, seed, replica0,
                       n_rep, block0, n_blk, out);
  }
  return hipGetLastError();
}

template <bool FP64>
static void launch_trajectory_t(int kind, const SetDev& sd, uint64_t replica,
                                int64_t n_steps, double* out_phi, double* out_v,
                                uint4* mt, hipStream_t st) {
  switch (kind) {
    case kOver:
      hipLaunchKernelGGL((trajectory_kernel<FP64, kOver>), dim3(1), dim3(64), 0, st, sd,
                         replica, n_steps, out_phi, out_v, mt);
      break;
    case kUnderSemiImplicit:
      hipLaunchKernelGGL((trajectory_kernel<FP64, kUnderSemiImplicit>), dim3(1), dim3(64), 0,
                         st, sd, replica, n_steps, out_phi, out_v, mt);
      break;
    default:
      hipLaunchKernelGGL((trajectory_kernel<FP64, kUnderExplicit>), dim3(1), dim3(64), 0, st,
                         sd, replica, n_steps, out_phi, out_v, mt);
  }
}

hipError_t launch_trajectory(bool fp64, int kind, const SetDev& sd,
                             uint64_t replica, int64_t n_steps, double* out_phi,
                             double* out_v, uint4* mt, hipStream_t st) {
  if (n_steps <= 0) return hipSuccess;
  if (fp64) {
    launch_trajectory_t<true>(kind, sd, replica, n_steps, out_phi, out_v, mt, st);
  } else {
    launch_trajectory_t<false>(kind, sd, replica, n_steps, out_phi, out_v, mt, st);
  }
  return hipGetLastError();
}

hipError_t launch_mt_words(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                           uint64_t block0, uint64_t n_blk, uint4* state,
                           uint32_t* out, hipStream_t st) {
  if (n_rep == 0 || n_blk == 0) return hipSuccess;
  hipLaunchKernelGGL(mt_words_kernel, dim3((uint32_t)((n_rep + 63) / 64)), dim3(64), 0, st,
                     seed, replica0, n_rep, block0, n_blk, state, out);
  return hipGetLastError();
}

}  // namespace fpt
