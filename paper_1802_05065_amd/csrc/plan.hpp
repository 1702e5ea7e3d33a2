// plan.hpp -- host-side state of an fpt_plan_t.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"

namespace fpt {

// Launches near the end of a refill run are this many times shorter.
constexpr int32_t kTailLaunchDivisor = 8;

// Workspace layout: byte offsets of the regions for `max_slots` lane-state
// slots.
struct WsLayout {
  uint64_t max_slots = 0;
  uint64_t off_sets = 0, off_chunks = 0, off_ctr = 0, off_mom = 0, off_hist = 0;
  uint64_t off_st_phi = 0, off_st_v = 0, off_st_j = 0, off_st_idx = 0, off_st_set = 0;
  uint64_t off_st_mt = 0;
  // second lane-state buffer for tail compaction (refill plans without MT)
  uint64_t off_alt_phi = 0, off_alt_v = 0, off_alt_j = 0, off_alt_idx = 0, off_alt_set = 0;
  bool has_alt = false;
  uint64_t off_group = 0;       // per-set positions of a regrouping (multi-set)
  uint64_t ws_bytes = 0;
};

struct Plan : WsLayout {
  std::vector<fpt_params> params;
  std::vector<SetDev> sets;     // derived constants, hist offsets
  std::vector<Chunk> chunks;    // multi-set work queue (64 replicas per entry)
  int precision = FPT_FP64;
  int model = kUnderExplicit;   // integrator kind
  bool multi = false;
  bool mt = false;              // FPT_RNG_MT19937: per-slot generator state
  fpt_tuning tuning_req{};      // as given (zeros: autotune)
  fpt_tuning tuning{};          // as used by the last simulate
  uint64_t total_replicas = 0;
  uint64_t total_flat = 0;      // size of the flat index space (with padding)
  uint64_t hist_bins = 0;
  int cus = 256;
  std::string arch = "gfx950";

  // the workspace layout (WsLayout) is sized for the largest launch shape;
  // a run in the library's static scratch lays it out for its own shape

  // last run
  uint64_t n_lanes = 0;
  uint64_t* hist_dev = nullptr;
  MomDev* ws_mom_ptr = nullptr;
  hipStream_t stream = nullptr;
  bool ran = false;
  fpt_run_stats stats{};

  // host resources (created lazily, on the first simulate)
  Counters* h_ctr = nullptr;    // pinned (a run in the static scratch points it
                                // at h_ctr_plain instead)
  Counters h_ctr_plain{};
  std::vector<SetDev> upload;   // set table as uploaded (sized with the plan)
  bool noalloc = false;         // the current run allocates nothing
  std::vector<hipEvent_t> events;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t graph_stream = nullptr;  // capture / replay stream of the graph path

  ~Plan();
  // lay out the workspace for `slots` lane-state slots (0: the largest shape)
  fpt_status layout(uint64_t slots = 0);
  SliceArgs slice_args(char* ws, uint64_t* hist, uint64_t n_lanes, int buf = 0) const;
  fpt_status maybe_compact(char* ws, SliceArgs& a, int& buf, uint64_t& lanes, int R,
                           hipStream_t st, bool* compacted);
  fpt_status enqueue_regroup(char* ws, const SliceArgs& a, int buf, uint64_t lanes, int R,
                             hipStream_t st);
  bool tail_launches(SliceArgs& a, uint64_t slots, uint64_t draw_per_group);
  bool tail_mode = false;
  uint64_t last_cursor = 0;     // cursor at the previous check
  uint64_t lanes_for(const fpt_tuning& t) const;
  // multi-set refill runs sort by set and refill between launches, and
  // refill only whole wavefronts inside one
  bool regroups(const fpt_tuning& t) const {
    return multi && has_alt && t.schedule == FPT_SCHED_REFILL && !t.no_regroup;
  }
  int resident_waves(int R) const;
  uint64_t launch_bound(uint64_t n_slots, int blocks) const;
  fpt_status ensure_host_resources(size_t n_events);
  fpt_status upload_sets(char* ws, const std::vector<SetDev>& table, hipStream_t st);
  fpt_status reset_run(char* ws, const SliceArgs& a, uint64_t n_lanes, int R, bool refill,
                       hipStream_t st);
  fpt_status resolve_tuning(char* ws, hipStream_t st);
  fpt_status simulate(void* workspace, int64_t* const* out_steps, uint64_t* out_hist,
                      hipStream_t st);
  // fpt_simulate in caller-independent scratch memory: `scratch` of
  // `scratch_bytes` (the library's static device array); no allocation
  fpt_status simulate_in_scratch(void* scratch, uint64_t scratch_bytes,
                                 int64_t* const* out_steps, uint64_t* out_hist,
                                 hipStream_t st);
  fpt_status histogram(int32_t set, uint64_t* host_counts, fpt_moments* host_m);
  fpt_status histogram_all(uint64_t* host_counts, fpt_moments* host_m);
  fpt_status run_stats(fpt_run_stats* out);
};

void fill_moments(const MomDev& m, double dt, fpt_moments* out);
fpt_status make_plan(const fpt_params* params, int32_t n_sets, int32_t precision,
                     const fpt_tuning* tuning, Plan** out);
const char* last_error();

}  // namespace fpt

// The C ABI's opaque plan handle.
struct fpt_plan_s {
  fpt::Plan* impl;
};
