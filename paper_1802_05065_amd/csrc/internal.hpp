// internal.hpp -- structures shared by the host runtime and the gfx950
// kernels of the first-passage-time library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpt.h"

namespace fpt {

constexpr int kWave = 64;          // wavefront width on CDNA
constexpr int kBlockThreads = 256; // threads per workgroup (4 wavefronts)
constexpr int kHistSlots = 1024;   // LDS hash entries for (set, bin) counts
constexpr int kMomSlots = 64;      // LDS hash entries for per-set moments
constexpr int kProbes = 32;        // linear-probe limit before the global path
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kInactive = 0xFFFFFFFFu;
constexpr int kChunk = 64;         // replicas per work-queue chunk
constexpr int kBinBits = 12;       // FPT_MAX_BINS = 1 << kBinBits
// Largest set count of a plan: every (set << kBinBits | bin) key, set index
// up to kMaxPlanSets - 1, stays below kEmpty, the LDS tables' empty marker.
constexpr int kMaxPlanSets = (1 << (32 - kBinBits)) - 1;
static_assert((uint64_t(kMaxPlanSets - 1) << kBinBits | ((1u << kBinBits) - 1)) < kEmpty,
              "histogram keys must not reach the empty marker");

// Integrator kinds (the kernel's MODEL template argument): the two models of
// fpt_model, plus the underdamped model with the semi-implicit scheme.
constexpr int kUnderExplicit = FPT_UNDERDAMPED;
constexpr int kOver = FPT_OVERDAMPED;
constexpr int kUnderSemiImplicit = 2;

inline int integrator_kind(const fpt_params& p) {
  if (p.model == FPT_OVERDAMPED) return kOver;
  return p.scheme == FPT_SEMI_IMPLICIT ? kUnderSemiImplicit : kUnderExplicit;
}

// Per-set constants, derived on the host (Algorithm 1 / 3 preamble).
struct alignas(16) SetDev {
  double gamma0, dgamma, dt, alpha, V0, sigma, th, phi0, v0;
  // FP32C constants (phase in revolutions, phi / 2 pi): bias term
  // G_k = gA + gB k in FP64, threshold, and FP32 step coefficients
  double gA, gB, th_rev;
  // (nkS_f = -kS; dG2_f, dG3_f = 2 and 3 bias increments; e0_f: initial
  // phase error, true phase = phr0_f + e0_f)
  float h_rev_f, damp_f, nkS_f, sig_f, dG_f, dG2_f, dG3_f, th_near_rev_f, phr0_f, e0_f, v0_f,
      pad_f;
  int64_t max_steps;    // klim
  uint64_t jmax;        // block of the last allowed step: (max_steps - 1) / 4
  int64_t k_hist;       // histogram covers steps [1, k_hist]
  double hist_scale;    // n_bins / k_hist (estimate of the bin, corrected exactly)
  uint64_t seed;
  uint64_t n_replicas;
  int64_t* out_steps;   // device, may be null
  uint64_t hist_off;    // first bin of this set in the histogram array
  uint32_t n_bins;
  uint32_t model;       // integrator kind
};

// A run of at most kChunk consecutive replicas of one set.
struct Chunk {
  uint32_t set;
  uint32_t count;
  uint64_t first;
};

// Per-set results in device memory (integers only).
struct alignas(16) MomDev {
  unsigned long long n_esc, n_cens, n_over, sum_k, sum_k2_lo, sum_k2_hi, pad0,
      pad1;
};

struct alignas(16) Counters {
  unsigned long long cursor;      // next flat replica index to hand out
  unsigned long long done;        // replicas finished (escaped or censored)
  unsigned long long lane_steps;  // lane-steps issued, idle lanes included
  unsigned long long compact;     // active slots found by a compaction pass
  unsigned long long extra_passes;  // multi-set blocks: passes beyond one per slot
  unsigned long long overflow;    // slots a move could not place (never expected)
  unsigned long long pad[2];
};

// Arguments of one integrator launch.
struct SliceArgs {
  const SetDev* sets;
  const Chunk* chunks;            // null: single set, flat index = replica
  unsigned long long chunk_mask;  // ring mask (server) or ~0 (plan)
  Counters* ctr;
  unsigned long long total;       // flat replicas that may be drawn
  unsigned long long* st_phi;     // resident lane state, slot = r*n_lanes+lane
  unsigned long long* st_v;
  unsigned long long* st_j;
  unsigned long long* st_idx;
  uint32_t* st_set;
  uint4* st_mt;                   // MT19937 state (156 groups per slot) or null
  unsigned long long n_lanes;
  unsigned long long* hist;
  MomDev* mom;
  int32_t blocks;                 // 4-step blocks in this launch
  int32_t refill;                 // 1: take new replicas as slots free up
  int32_t clamp;                  // 1: cursor may not pass `total` (server)
  int32_t whole_waves;            // 1: refill only wavefronts whose slot is free
                                  // in every lane (multi-set runs that sort by set
                                  // and refill between launches)
};

}  // namespace fpt
