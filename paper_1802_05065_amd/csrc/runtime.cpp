// runtime.cpp -- plans: validation and per-set constants, workspace layout,
// the launch loop of fpt_simulate, histogram / moment readout, diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "autotune.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace fpt {

namespace {
thread_local std::string g_error;
}

fpt_status fail(fpt_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

void clear_error() { g_error.clear(); }

const char* last_error() { return g_error.c_str(); }

static bool finite_or_nan(double x) { return std::isfinite(x) || std::isnan(x); }

fpt_status validate_params(const fpt_params& p, int i) {
  if (p.model != FPT_UNDERDAMPED && p.model != FPT_OVERDAMPED)
    return fail(FPT_E_INVAL, "set %d: model %d is not 0 (underdamped) or 1 (overdamped)", i,
                p.model);
  if (p.scheme != FPT_EXPLICIT && p.scheme != FPT_SEMI_IMPLICIT)
    return fail(FPT_E_INVAL, "set %d: scheme %d is not 0 (explicit) or 1 (semi-implicit)", i,
                p.scheme);
  if (p.model == FPT_OVERDAMPED && p.scheme != FPT_EXPLICIT)
    return fail(FPT_E_INVAL, "set %d: the overdamped model has only scheme 0", i);
  if (p.rng != FPT_RNG_PHILOX && p.rng != FPT_RNG_MT19937)
    return fail(FPT_E_INVAL, "set %d: rng %d is not 0 (Philox) or 1 (MT19937)", i, p.rng);
  if (p.n_bins < 1 || p.n_bins > FPT_MAX_BINS)
    return fail(FPT_E_INVAL, "set %d: n_bins %d outside [1, %d]", i, p.n_bins, FPT_MAX_BINS);
  if (!(p.dt > 0.0) || !std::isfinite(p.dt))
    return fail(FPT_E_INVAL, "set %d: dt must be finite and > 0", i);
  if (!(p.T >= 0.0) || !std::isfinite(p.T))
    return fail(FPT_E_INVAL, "set %d: T must be finite and >= 0", i);
  if (!std::isfinite(p.alpha) || (p.model == FPT_UNDERDAMPED && p.alpha < 0.0))
    return fail(FPT_E_INVAL, "set %d: alpha must be finite and >= 0", i);
  if (!std::isfinite(p.V0) || !std::isfinite(p.gamma0) || !std::isfinite(p.ramp))
    return fail(FPT_E_INVAL, "set %d: V0, gamma0 and ramp must be finite", i);
  if (!finite_or_nan(p.phi0) || !finite_or_nan(p.v0) || !finite_or_nan(p.threshold))
    return fail(FPT_E_INVAL, "set %d: phi0, v0, threshold must be finite or NaN", i);
  if (std::isnan(p.phi0) && p.model == FPT_UNDERDAMPED && !(std::fabs(p.gamma0) <= 1.0))
    return fail(FPT_E_INVAL, "set %d: default phi0 = arcsin(gamma0) needs |gamma0| <= 1", i);
  if (std::isnan(p.phi0) && p.model == FPT_OVERDAMPED &&
      !(p.V0 != 0.0 && std::fabs(p.gamma0 / p.V0) <= 1.0))
    return fail(FPT_E_INVAL,
                "set %d: default phi0 = arcsin(gamma0 / V0) needs V0 != 0 and |gamma0| <= |V0|",
                i);
  if (p.max_steps < 1 || p.max_steps > (int64_t(1) << 50))
    return fail(FPT_E_INVAL, "set %d: max_steps %lld outside [1, 2^50]", i,
                (long long)p.max_steps);
  if (p.n_replicas < 0 || p.n_replicas > (int64_t(1) << 48))
    return fail(FPT_E_INVAL, "set %d: n_replicas %lld outside [0, 2^48]", i,
                (long long)p.n_replicas);
  if (p.hist_k_max < 0 || p.hist_k_max > (int64_t(1) << 50))
    return fail(FPT_E_INVAL, "set %d: hist_k_max outside [0, 2^50]", i);
  return FPT_OK;
}

static float round_toward_minus_inf(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -INFINITY);
  return f;
}

SetDev derive_set(const fpt_params& p) {
  SetDev s;
  std::memset(&s, 0, sizeof(s));
  s.gamma0 = p.gamma0;
  s.dgamma = p.ramp * p.dt;  // delta-gamma of Algorithm 3
  s.dt = p.dt;
  s.alpha = p.alpha;
  s.V0 = p.V0;
  if (p.model == FPT_UNDERDAMPED) {
    const double D = p.alpha * p.T;  // D = beta theta, Eq. (9)
    s.sigma = std::sqrt(2.0 * D * p.dt);
  } else {
    s.sigma = std::sqrt(2.0 * p.T * p.dt);
  }
  // default start: the bottom of the well, arcsin(gamma0) for Eq. (10) (V0
  // multiplies the bias too), arcsin(gamma0 / V0) for the overdamped
  // potential -V0 cos(phi) - gamma phi
  const double well_sin = p.model == FPT_UNDERDAMPED ? p.gamma0 : p.gamma0 / p.V0;
  s.phi0 = std::isnan(p.phi0) ? std::asin(well_sin) : p.phi0;
  s.v0 = std::isnan(p.v0) ? 0.0 : p.v0;
  // default threshold: top of the washboard barrier, pi - arcsin(gamma)
  s.th = std::isnan(p.threshold) ? 3.14159265358979323846 - s.phi0 : p.threshold;
  // FP32C: phase in revolutions so v_sin_f32 takes it directly; the
  // Box-Muller constant sqrt(2 ln 2) goes into the noise scale
  const double twopi = 2.0 * 3.14159265358979323846;
  const double sqrt2ln2 = 1.1774100225154747;
  if (p.model == FPT_UNDERDAMPED) {
    s.gA = p.dt * p.V0 * p.gamma0;     // G_k = h V0 gamma_k
    s.gB = p.dt * p.V0 * s.dgamma;
    s.nkS_f = (float)(-p.dt * p.V0);
    s.sig_f = (float)(s.sigma * sqrt2ln2);
    s.h_rev_f = (float)(p.dt / twopi);
    s.damp_f = (float)(1.0 - p.dt * p.alpha);
  } else {
    s.gA = p.dt * p.gamma0 / twopi;    // G_k = h gamma_k / 2 pi
    s.gB = p.dt * s.dgamma / twopi;
    s.nkS_f = (float)(-p.dt * p.V0 / twopi);
    s.sig_f = (float)(s.sigma * sqrt2ln2 / twopi);
    s.h_rev_f = 0.0f;
    s.damp_f = 1.0f;
  }
  s.dG_f = (float)s.gB;
  s.dG2_f = (float)(2.0 * s.gB);
  s.dG3_f = (float)(3.0 * s.gB);
  s.th_rev = s.th / twopi;
  // at or below th_near_rev_f the compensated phase cannot exceed th_rev:
  // 8 float ulps of margin cover the compensation term and the rounding
  float tn = round_toward_minus_inf(s.th_rev);
  for (int i = 0; i < 8; ++i) tn = std::nextafter(tn, -INFINITY);
  s.th_near_rev_f = tn;
  const double phr0 = s.phi0 / twopi;
  s.phr0_f = (float)phr0;
  s.e0_f = (float)(phr0 - (double)s.phr0_f);
  s.v0_f = (float)s.v0;
  s.max_steps = p.max_steps;
  s.jmax = (uint64_t)(p.max_steps - 1) / 4;
  s.k_hist = p.hist_k_max > 0 ? p.hist_k_max : p.max_steps;
  s.hist_scale = (double)p.n_bins / (double)s.k_hist;
  s.seed = p.seed;
  s.n_replicas = (uint64_t)p.n_replicas;
  s.out_steps = nullptr;
  s.hist_off = 0;
  s.n_bins = (uint32_t)p.n_bins;
  s.model = (uint32_t)integrator_kind(p);
  return s;
}

DeviceInfo device_info() {
  DeviceInfo d;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
    (void)hipGetLastError();
    return d;
  }
  if (hipGetDevice(&d.device) != hipSuccess) return d;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d.device) ==
          hipSuccess &&
      cus > 0)
    d.cus = cus;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d.device) == hipSuccess) {
    std::string a = prop.gcnArchName;
    d.arch = a.substr(0, a.find(':'));
  }
  return d;
}

// ---------------------------------------------------------------------------
// Plans

// FPT_VERBOSE=1 prints run-time decisions (tail mode, compactions) to stderr.
static bool verbose() {
  const char* v = std::getenv("FPT_VERBOSE");
  return v && v[0] == '1';
}

static uint64_t align256(uint64_t x) { return round_up(x, 256); }

fpt_status Plan::layout(uint64_t slots) {
  if (slots == 0) {
    const DeviceInfo di = device_info();
    cus = di.cus;
    arch = di.arch;
    const uint64_t max_r = mt ? 1 : kMaxReplicasPerLane;
    if (tuning_req.schedule == FPT_SCHED_ONE_PER_LANE) {
      slots = round_up(std::max<uint64_t>(total_flat, 1), kBlockThreads * max_r);
    } else {
      slots = (uint64_t)cus * 4 * kMaxWavesPerSimd * kWave * max_r;
    }
  }
  max_slots = slots;
  uint64_t off = 0;
  off_sets = off;
  off = align256(off + sizeof(SetDev) * sets.size());
  off_chunks = off;
  off = align256(off + sizeof(Chunk) * chunks.size());
  off_ctr = off;
  off = align256(off + sizeof(Counters));
  off_mom = off;
  off = align256(off + sizeof(MomDev) * sets.size());
  off_hist = off;
  off = align256(off + sizeof(uint64_t) * std::max<uint64_t>(hist_bins, 1));
  off_st_phi = off;
  off = align256(off + 8 * slots);
  off_st_v = off;
  off = align256(off + 8 * slots);
  off_st_j = off;
  off = align256(off + 8 * slots);
  off_st_idx = off;
  off = align256(off + 8 * slots);
  off_st_set = off;
  off = align256(off + 4 * slots);
  off_st_mt = off;
  if (mt) off = align256(off + sizeof(uint4) * kMtGroupsPerSlot * slots);
  has_alt = !mt && tuning_req.schedule == FPT_SCHED_REFILL;
  if (has_alt) {
    off_alt_phi = off;
    off = align256(off + 8 * slots);
    off_alt_v = off;
    off = align256(off + 8 * slots);
    off_alt_j = off;
    off = align256(off + 8 * slots);
    off_alt_idx = off;
    off = align256(off + 8 * slots);
    off_alt_set = off;
    off = align256(off + 4 * slots);
    off_group = off;  // per-set counts, then per-set first positions
    if (multi) off = align256(off + 2 * sizeof(unsigned long long) * sets.size());
  }
  ws_bytes = off;
  return FPT_OK;
}

SliceArgs Plan::slice_args(char* ws, uint64_t* hist, uint64_t lanes, int buf) const {
  SliceArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sets = reinterpret_cast<const SetDev*>(ws + off_sets);
  a.chunks = multi ? reinterpret_cast<const Chunk*>(ws + off_chunks) : nullptr;
  a.chunk_mask = ~0ull;
  a.ctr = reinterpret_cast<Counters*>(ws + off_ctr);
  a.total = total_flat;
  a.st_phi = reinterpret_cast<unsigned long long*>(ws + off_st_phi);
  a.st_v = reinterpret_cast<unsigned long long*>(ws + off_st_v);
  a.st_j = reinterpret_cast<unsigned long long*>(ws + off_st_j);
  a.st_idx = reinterpret_cast<unsigned long long*>(ws + off_st_idx);
  a.st_set = reinterpret_cast<uint32_t*>(ws + off_st_set);
  if (buf == 1 && has_alt) {
    a.st_phi = reinterpret_cast<unsigned long long*>(ws + off_alt_phi);
    a.st_v = reinterpret_cast<unsigned long long*>(ws + off_alt_v);
    a.st_j = reinterpret_cast<unsigned long long*>(ws + off_alt_j);
    a.st_idx = reinterpret_cast<unsigned long long*>(ws + off_alt_idx);
    a.st_set = reinterpret_cast<uint32_t*>(ws + off_alt_set);
  }
  a.st_mt = mt ? reinterpret_cast<uint4*>(ws + off_st_mt) : nullptr;
  a.n_lanes = lanes;
  a.hist = reinterpret_cast<unsigned long long*>(hist);
  a.mom = reinterpret_cast<MomDev*>(ws + off_mom);
  a.blocks = 0;
  a.refill = 0;
  a.clamp = 0;
  return a;
}

uint64_t Plan::lanes_for(const fpt_tuning& t) const {
  const uint64_t R = (uint64_t)t.replicas_per_lane;
  if (t.schedule == FPT_SCHED_ONE_PER_LANE)
    return round_up((std::max<uint64_t>(total_flat, 1) + R - 1) / R, kBlockThreads);
  uint64_t lanes = (uint64_t)cus * 4 * (uint64_t)t.waves_per_simd * kWave;
  const uint64_t need = round_up((total_flat + R - 1) / R, kBlockThreads);
  return std::max<uint64_t>(std::min(lanes, need), kBlockThreads);
}

Plan::~Plan() {
  if (h_ctr) (void)hipHostFree(h_ctr);
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph_stream) (void)hipStreamDestroy(graph_stream);
}

fpt_status Plan::ensure_host_resources(size_t n_events) {
  if (!h_ctr) FPT_HIP(hipHostMalloc((void**)&h_ctr, sizeof(Counters), hipHostMallocDefault));
  while (events.size() < n_events) {
    hipEvent_t e;
    FPT_HIP(hipEventCreate(&e));
    events.push_back(e);
  }
  return FPT_OK;
}

// Reset counters, results and lane state, then bind every slot's first
// replica.  `sets_dev` already holds the set table.
fpt_status Plan::reset_run(char* ws, const SliceArgs& a, uint64_t lanes, int R, bool refill,
                           hipStream_t st) {
  FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(a.ctr),
                          sizeof(Counters) / 8, 0ull, st));
  FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(a.mom),
                          sizeof(MomDev) / 8 * sets.size(), 0ull, st));
  FPT_HIP(launch_fill_u64(a.hist, hist_bins, 0ull, st));
  if (multi && has_alt)  // the regroup's per-set counts
    FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(ws + off_group), sets.size(),
                            0ull, st));
  const uint64_t n_slots = lanes * (uint64_t)R;
  const uint64_t n_assign = std::min<uint64_t>(n_slots, total_flat);
  FPT_HIP(launch_init(precision == FPT_FP64, a, n_slots, n_assign, st));
  if (refill) FPT_HIP(launch_fill_u64(&a.ctr->cursor, 1, n_assign, st));
  return FPT_OK;
}

fpt_status Plan::upload_sets(char* ws, const std::vector<SetDev>& table,
                             hipStream_t st) {
  FPT_HIP(hipMemcpyAsync(ws + off_sets, table.data(), sizeof(SetDev) * table.size(),
                         hipMemcpyHostToDevice, st));
  if (multi && !chunks.empty())
    FPT_HIP(hipMemcpyAsync(ws + off_chunks, chunks.data(), sizeof(Chunk) * chunks.size(),
                           hipMemcpyHostToDevice, st));
  return FPT_OK;
}

// Upper bound on launches: no replica needs more than jmax+1 blocks, and all
// replicas together cannot need more than their summed blocks spread over the
// slots, plus the longest single replica for the tail.  A multi-set run
// counts every work-queue chunk as 64 replicas: a wavefront that takes a
// chunk may keep all its lanes until the chunk's last replica is done.
uint64_t Plan::launch_bound(uint64_t n_slots, int blocks) const {
  uint64_t longest = 0;
  long double work = 0;
  for (const SetDev& s : sets) {
    longest = std::max<uint64_t>(longest, s.jmax + 1);
    const uint64_t n = multi ? round_up(s.n_replicas, (uint64_t)kChunk) : s.n_replicas;
    work += (long double)n * (long double)(s.jmax + 1);
  }
  const long double per_launch = (long double)n_slots * (long double)blocks;
  const uint64_t spread = (uint64_t)(work / per_launch) + 1;
  return 2 * (spread + longest / (uint64_t)blocks + 1) + 16;
}

// When fewer undrawn replicas are left than there are slots, or will be
// after the next group of launches at the cursor's last rate of advance (and
// compaction is on), the run checks for compaction after every launch and
// launches an eighth as many steps, so the launch width can follow the decay
// of the active replicas from the moment the queue drains.  Returns true
// when it changes the launches.
bool Plan::tail_launches(SliceArgs& a, uint64_t slots, uint64_t draw_per_group) {
  if (!has_alt || tuning.no_compaction || !a.refill ||
      h_ctr->cursor + slots + draw_per_group < total_flat)
    return false;
  const int32_t shorter = std::max<int32_t>(16, a.blocks / kTailLaunchDivisor);
  if (tail_mode || shorter == a.blocks) return false;
  tail_mode = true;
  if (verbose())
    std::fprintf(stderr, "[fpt] tail: %lld undrawn, %llu slots, launches %d -> %d blocks\n",
                 (long long)total_flat - (long long)h_ctr->cursor, (unsigned long long)slots,
                 a.blocks, shorter);
  a.blocks = shorter;
  return true;
}

// Tail compaction between launches (the counters in h_ctr are current): when
// no undrawn replica is left and the active ones fill at most 80% of the
// slots, count them, and if the launch can narrow by a tenth or more, move
// their state to a dense prefix of the other state buffer (in set order for
// multi-set plans).  (Thresholds from a sweep on the uneven and batched
// workloads: 50%/25% left 8% of the batched run's lane-steps idle, 80%/10%
// leaves 3%.)
constexpr uint64_t kCompactTriggerPercent = 80;
constexpr uint64_t kCompactNarrowPercent = 90;

fpt_status Plan::maybe_compact(char* ws, SliceArgs& a, int& buf, uint64_t& lanes, int R,
                               hipStream_t st, bool* compacted) {
  *compacted = false;
  if (!has_alt || tuning.no_compaction || !a.refill) return FPT_OK;
  if (h_ctr->cursor < total_flat || lanes <= (uint64_t)kBlockThreads) return FPT_OK;
  const uint64_t slots = lanes * (uint64_t)R;
  const uint64_t done = (uint64_t)h_ctr->done;
  const uint64_t active_bound = total_flat - std::min<uint64_t>(done, total_flat);
  if (active_bound * 100 > slots * kCompactTriggerPercent) return FPT_OK;
  auto* counts = reinterpret_cast<unsigned long long*>(ws + off_group);
  auto* first = counts + sets.size();
  FPT_HIP(launch_fill_u64(&a.ctr->compact, 1, 0ull, st));
  if (multi) {
    FPT_HIP(launch_group_count(a, slots, counts, first, sets.size(), st));
  } else {
    FPT_HIP(launch_compact_count(a, slots, st));
  }
  FPT_HIP(hipMemcpyAsync(h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  FPT_HIP(hipStreamSynchronize(st));
  const uint64_t active = h_ctr->compact;
  const uint64_t new_lanes = std::max<uint64_t>(
      kBlockThreads, round_up((active + (uint64_t)R - 1) / (uint64_t)R, kBlockThreads));
  if (new_lanes * 100 > lanes * kCompactNarrowPercent) return FPT_OK;
  SliceArgs dst = slice_args(ws, reinterpret_cast<uint64_t*>(a.hist), new_lanes, 1 - buf);
  dst.blocks = a.blocks;
  dst.refill = a.refill;
  dst.clamp = a.clamp;
  dst.whole_waves = a.whole_waves;
  if (multi) {
    FPT_HIP(launch_group_move(a, dst, slots, new_lanes * (uint64_t)R, first, st));
  } else {
    FPT_HIP(launch_fill_u64(&a.ctr->compact, 1, 0ull, st));
    FPT_HIP(launch_compact_move(a, dst, slots, new_lanes * (uint64_t)R, st));
  }
  if (verbose())
    std::fprintf(stderr, "[fpt] compaction: %llu active slots, %llu -> %llu lanes\n",
                 (unsigned long long)active, (unsigned long long)lanes,
                 (unsigned long long)new_lanes);
  a = dst;
  buf = 1 - buf;
  lanes = new_lanes;
  ++stats.n_compactions;
  *compacted = true;
  return FPT_OK;
}

// Multi-set refill runs, after every launch while undrawn replicas are left:
// the active slots move into set order through the other state buffer, the
// free slots past them take the next replicas in queue order, and the state
// comes back, so wavefronts hold one set again (inside a launch only
// wavefronts free in every lane draw new replicas).  Six small kernels, no
// host synchronization, so a captured group of launches includes them.
// (The per-set counts they use are zero at the start of a run and after
// every count.)
fpt_status Plan::enqueue_regroup(char* ws, const SliceArgs& a, int buf, uint64_t lanes, int R,
                                 hipStream_t st) {
  const uint64_t slots = lanes * (uint64_t)R;
  const SliceArgs other = slice_args(ws, reinterpret_cast<uint64_t*>(a.hist), lanes, 1 - buf);
  auto* counts = reinterpret_cast<unsigned long long*>(ws + off_group);
  auto* first = counts + sets.size();
  FPT_HIP(launch_group_count(a, slots, counts, first, sets.size(), st));
  FPT_HIP(launch_group_move(a, other, slots, slots, first, st));
  FPT_HIP(launch_group_refill(precision == FPT_FP64, other, slots, st));
  FPT_HIP(launch_copy_state(other, a, slots, true, st));
  return FPT_OK;
}

fpt_status Plan::simulate(void* workspace, int64_t* const* out_steps,
                          uint64_t* out_hist, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  char* ws = static_cast<char*>(workspace);
  if (!ws) return fail(FPT_E_INVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(FPT_E_INVAL, "workspace must be 256-byte aligned");
  hist_dev = out_hist ? out_hist : reinterpret_cast<uint64_t*>(ws + off_hist);
  ws_mom_ptr = reinterpret_cast<MomDev*>(ws + off_mom);
  ran = false;
  stream = st;

  if (!noalloc) FPT_TRY(resolve_tuning(ws, st));  // the scratch run set `tuning` itself
  const int R = tuning.replicas_per_lane;
  const bool refill = tuning.schedule == FPT_SCHED_REFILL;
  n_lanes = lanes_for(tuning);
  const uint64_t n_slots = n_lanes * (uint64_t)R;
  if (n_slots > max_slots)
    return fail(FPT_E_INVAL, "launch shape needs %llu slots, workspace holds %llu",
                (unsigned long long)n_slots, (unsigned long long)max_slots);
  const int blocks = tuning.steps_per_launch / 4;

  // the uploaded table (sized with the plan) carries this call's outputs
  for (size_t i = 0; i < sets.size(); ++i) {
    upload[i] = sets[i];
    upload[i].out_steps = out_steps ? out_steps[i] : nullptr;
  }
  FPT_TRY(upload_sets(ws, upload, st));

  // multi-set refill runs keep wavefronts to one set (enqueue_regroup)
  const bool regroup = regroups(tuning);
  SliceArgs a = slice_args(ws, hist_dev, n_lanes);
  a.blocks = blocks;
  a.refill = refill ? 1 : 0;
  a.whole_waves = regroup ? 1 : 0;
  FPT_TRY(reset_run(ws, a, n_lanes, R, refill, st));

  uint64_t lanes = n_lanes;  // narrows at each tail compaction
  int buf = 0;
  tail_mode = false;
  last_cursor = std::min<uint64_t>(n_slots, total_flat);  // the cursor after reset_run
  const bool fp64 = precision == FPT_FP64;
  // the bound is on 4-step blocks issued, so shorter tail launches count less
  const uint64_t bound_blocks = launch_bound(n_slots, blocks) * (uint64_t)blocks;
  uint64_t blocks_issued = 0;
  stats = fpt_run_stats{};
  stats.tuning = tuning;
  int group = 1;
  int64_t launches = 0;
  double kernel_ms = 0.0;
  bool finished = total_replicas == 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;
  size_t ev_used = 0;

  if (tuning.use_graph && !finished) {
    // A fixed group of launches plus the status copy is captured on a
    // plan-owned stream (the legacy NULL stream cannot be captured) and
    // replayed; events order it after earlier work on `st` and order later
    // work on `st` after it.  A tail compaction changes the launch width,
    // so the graph is captured again after one.
    group = 8;
    FPT_TRY(ensure_host_resources(4));
    if (!graph_stream) FPT_HIP(hipStreamCreateWithFlags(&graph_stream, hipStreamNonBlocking));
    FPT_HIP(hipEventRecord(events[2], st));
    FPT_HIP(hipStreamWaitEvent(graph_stream, events[2], 0));
    bool graph_regroup = false;  // the captured group regroups after each launch
    auto capture = [&]() -> fpt_status {
      if (graph_exec) {
        (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
      }
      graph_regroup = regroup && last_cursor < total_flat;
      const uint32_t groups = (uint32_t)(lanes / kBlockThreads);
      hipGraph_t g = nullptr;
      FPT_HIP(hipStreamBeginCapture(graph_stream, hipStreamCaptureModeThreadLocal));
      hipError_t cap_err = hipSuccess;
      for (int i = 0; i < group && cap_err == hipSuccess; ++i) {
        cap_err = launch_slice(fp64, model, R, multi, a, groups, graph_stream);
        if (cap_err == hipSuccess && graph_regroup &&
            enqueue_regroup(ws, a, buf, lanes, R, graph_stream) != FPT_OK)
          cap_err = hipErrorUnknown;
      }
      if (cap_err == hipSuccess)
        cap_err = hipMemcpyAsync(h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost,
                                 graph_stream);
      hipError_t end_err = hipStreamEndCapture(graph_stream, &g);
      if (cap_err != hipSuccess || end_err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(FPT_E_DEVICE, "graph capture failed: %s",
                    hipGetErrorString(cap_err != hipSuccess ? cap_err : end_err));
      }
      hipError_t inst = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (inst != hipSuccess)
        return fail(FPT_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(inst));
      return FPT_OK;
    };
    FPT_TRY(capture());
    while (!finished) {
      FPT_HIP(hipEventRecord(events[0], graph_stream));
      FPT_HIP(hipGraphLaunch(graph_exec, graph_stream));
      FPT_HIP(hipEventRecord(events[1], graph_stream));
      FPT_HIP(hipEventSynchronize(events[1]));
      float ms = 0.f;
      FPT_HIP(hipEventElapsedTime(&ms, events[0], events[1]));
      kernel_ms += ms;
      launches += group;
      if (graph_regroup) stats.n_regroups += group;
      blocks_issued += (uint64_t)group * (uint64_t)a.blocks;
      if (h_ctr->overflow)
        return fail(FPT_E_DEVICE, "regroup could not place %llu slots",
                    (unsigned long long)h_ctr->overflow);
      finished = h_ctr->done >= total_replicas;
      if (!finished && blocks_issued > bound_blocks)
        return fail(FPT_E_DEVICE, "run did not finish within %llu steps per slot",
                    (unsigned long long)(4 * bound_blocks));
      const uint64_t advance = h_ctr->cursor - std::min<uint64_t>(h_ctr->cursor, last_cursor);
      last_cursor = h_ctr->cursor;
      if (!finished) {
        bool compacted = false;
        FPT_TRY(maybe_compact(ws, a, buf, lanes, R, graph_stream, &compacted));
        const bool shorter = tail_launches(a, lanes * (uint64_t)R, advance);
        if (shorter) group = 1;
        const bool drained = graph_regroup && last_cursor >= total_flat;
        if (compacted || shorter || drained) FPT_TRY(capture());
      }
    }
    FPT_HIP(hipEventRecord(events[3], graph_stream));
    FPT_HIP(hipStreamWaitEvent(st, events[3], 0));
  } else {
    // a run in the static scratch creates no events: it waits on the stream
    // and leaves kernel_ms at 0
    if (!noalloc) marks.reserve(16);
    while (!finished) {
      if (!noalloc) FPT_TRY(ensure_host_resources(ev_used + 2 * group + 1));
      const uint32_t groups = (uint32_t)(lanes / kBlockThreads);
      const bool regroup_now = regroup && last_cursor < total_flat;
      for (int i = 0; i < group; ++i) {
        if (noalloc) {
          FPT_HIP(launch_slice(fp64, model, R, multi, a, groups, st));
        } else {
          hipEvent_t e0 = events[ev_used++], e1 = events[ev_used++];
          FPT_HIP(hipEventRecord(e0, st));
          FPT_HIP(launch_slice(fp64, model, R, multi, a, groups, st));
          FPT_HIP(hipEventRecord(e1, st));
          marks.emplace_back(e0, e1);
        }
        if (regroup_now) {
          FPT_TRY(enqueue_regroup(ws, a, buf, lanes, R, st));
          ++stats.n_regroups;
        }
        ++launches;
        blocks_issued += (uint64_t)a.blocks;
      }
      FPT_HIP(hipMemcpyAsync(h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
      if (noalloc) {
        FPT_HIP(hipStreamSynchronize(st));
      } else {
        hipEvent_t sync = events[ev_used++];
        FPT_HIP(hipEventRecord(sync, st));
        FPT_HIP(hipEventSynchronize(sync));
      }
      for (auto& m : marks) {
        float ms = 0.f;
        FPT_HIP(hipEventElapsedTime(&ms, m.first, m.second));
        kernel_ms += ms;
      }
      marks.clear();
      ev_used = 0;
      if (h_ctr->overflow)
        return fail(FPT_E_DEVICE, "regroup could not place %llu slots",
                    (unsigned long long)h_ctr->overflow);
      finished = h_ctr->done >= total_replicas;
      if (!finished && blocks_issued > bound_blocks)
        return fail(FPT_E_DEVICE, "run did not finish within %llu steps per slot",
                    (unsigned long long)(4 * bound_blocks));
      const uint64_t advance = h_ctr->cursor - std::min<uint64_t>(h_ctr->cursor, last_cursor);
      const uint64_t per_launch = advance / (uint64_t)group;
      last_cursor = h_ctr->cursor;
      if (!finished) {
        bool compacted = false;
        FPT_TRY(maybe_compact(ws, a, buf, lanes, R, st, &compacted));
      }
      group = std::min(group * 2, 8);
      if (!finished &&
          (tail_mode || tail_launches(a, lanes * (uint64_t)R, per_launch * (uint64_t)group)))
        group = 1;
    }
  }
  if (total_replicas == 0 && !noalloc) FPT_TRY(ensure_host_resources(1));
  if (total_replicas > 0) {
    stats.lane_steps = h_ctr->lane_steps;
    stats.extra_passes = h_ctr->extra_passes;
  }
  stats.n_launches = launches;
  stats.kernel_ms = kernel_ms;
  stats.wall_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
          .count();
  ran = true;
  return FPT_OK;
}

// fpt_simulate without any allocation: the workspace is `scratch` (the
// library's static device array of `scratch_bytes`), laid out for this
// call's own launch shape instead of the largest one.  The tuning must be
// complete (no autotuning trials) and graph-free; the counters come back
// through plan-owned host memory and no events are created.
fpt_status Plan::simulate_in_scratch(void* scratch, uint64_t scratch_bytes,
                                     int64_t* const* out_steps, uint64_t* out_hist,
                                     hipStream_t st) {
  const fpt_tuning& t = tuning_req;
  if (t.replicas_per_lane == 0 || t.waves_per_simd == 0 || t.steps_per_launch == 0)
    return fail(FPT_E_INVAL,
                "the allocation-free run needs a complete tuning (replicas_per_lane, "
                "waves_per_simd, steps_per_launch): it runs no autotuning trials");
  if (t.use_graph)
    return fail(FPT_E_INVAL, "the allocation-free run does not replay graphs (use_graph 0)");
  fpt_tuning used = t;
  used.waves_per_simd = std::min(used.waves_per_simd, resident_waves(used.replicas_per_lane));
  const uint64_t slots = lanes_for(used) * (uint64_t)used.replicas_per_lane;
  const WsLayout full = *this;
  FPT_TRY(layout(slots));
  if (ws_bytes > scratch_bytes) {
    const uint64_t need = ws_bytes;
    static_cast<WsLayout&>(*this) = full;
    return fail(FPT_E_NOMEM,
                "the plan needs %llu bytes of workspace at its launch shape; the library's "
                "static scratch holds %llu (use fpt_simulate with a workspace)",
                (unsigned long long)need, (unsigned long long)scratch_bytes);
  }
  Counters* pinned = h_ctr;
  h_ctr = &h_ctr_plain;
  noalloc = true;
  tuning = used;
  const fpt_status res = simulate(scratch, out_steps, out_hist, st);
  noalloc = false;
  h_ctr = pinned;
  static_cast<WsLayout&>(*this) = full;
  return res;
}

fpt_status Plan::histogram(int32_t set, uint64_t* host_counts, fpt_moments* host_m) {
  if (!ran) return fail(FPT_E_STATE, "fpt_histogram before a finished fpt_simulate");
  if (set < 0 || set >= (int32_t)sets.size())
    return fail(FPT_E_INVAL, "set %d outside [0, %zu)", set, sets.size());
  FPT_HIP(hipStreamSynchronize(stream));
  const SetDev& s = sets[(size_t)set];
  if (host_counts)
    FPT_HIP(hipMemcpy(host_counts, hist_dev + s.hist_off, sizeof(uint64_t) * s.n_bins,
                      hipMemcpyDeviceToHost));
  if (host_m) {
    MomDev m;
    FPT_HIP(hipMemcpy(&m, ws_mom_ptr + set, sizeof(MomDev), hipMemcpyDeviceToHost));
    fill_moments(m, s.dt, host_m);
  }
  return FPT_OK;
}

fpt_status Plan::histogram_all(uint64_t* host_counts, fpt_moments* host_m) {
  if (!ran) return fail(FPT_E_STATE, "fpt_histogram_all before a finished fpt_simulate");
  FPT_HIP(hipStreamSynchronize(stream));
  if (host_counts && hist_bins > 0)
    FPT_HIP(hipMemcpy(host_counts, hist_dev, sizeof(uint64_t) * hist_bins,
                      hipMemcpyDeviceToHost));
  if (host_m && !sets.empty()) {
    std::vector<MomDev> m(sets.size());
    FPT_HIP(hipMemcpy(m.data(), ws_mom_ptr, sizeof(MomDev) * sets.size(),
                      hipMemcpyDeviceToHost));
    for (size_t i = 0; i < sets.size(); ++i) fill_moments(m[i], sets[i].dt, &host_m[i]);
  }
  return FPT_OK;
}

void fill_moments(const MomDev& m, double dt, fpt_moments* out) {
  out->n_escaped = m.n_esc;
  out->n_censored = m.n_cens;
  out->n_overflow = m.n_over;
  out->sum_k = m.sum_k;
  out->sum_k2_lo = m.sum_k2_lo;
  out->sum_k2_hi = m.sum_k2_hi;
  out->mean_t = NAN;
  out->se_t = NAN;
  const uint64_t n = m.n_esc;
  if (n > 0) out->mean_t = dt * ((double)m.sum_k / (double)n);
  if (n > 1) {
    const unsigned __int128 k2 = ((unsigned __int128)m.sum_k2_hi << 64) | m.sum_k2_lo;
    const unsigned __int128 m2 =
        (unsigned __int128)n * k2 - (unsigned __int128)m.sum_k * (unsigned __int128)m.sum_k;
    out->se_t = dt * std::sqrt((double)m2 / ((double)n * (double)n * (double)(n - 1)));
  }
}

fpt_status Plan::run_stats(fpt_run_stats* out) {
  if (!ran) return fail(FPT_E_STATE, "fpt_plan_stats before a finished fpt_simulate");
  FPT_HIP(hipStreamSynchronize(stream));
  uint64_t rs = 0;
  std::vector<MomDev> m(sets.size());
  if (!sets.empty())
    FPT_HIP(hipMemcpy(m.data(), ws_mom_ptr, sizeof(MomDev) * sets.size(),
                      hipMemcpyDeviceToHost));
  for (size_t i = 0; i < sets.size(); ++i)
    rs += m[i].sum_k + m[i].n_cens * (uint64_t)sets[i].max_steps;
  *out = stats;
  out->replica_steps = rs;
  return FPT_OK;
}

// Scheduling estimate of a replica's steps (only orders the work queue): a
// ramped bias switches by the time it reaches 1, (1 - gamma0) / (ramp dt)
// steps; a fixed bias below 1 escapes at the Kramers rate
// omega / (2 pi) exp(-dU / T), omega = sqrt(V0) (1 - gamma^2)^(1/4) and
// dU = 2 V0 (sqrt(1 - gamma^2) - gamma arccos gamma); at most max_steps.
static double expected_steps(const fpt_params& q) {
  const double cap = (double)q.max_steps;
  const double dgamma = q.ramp * q.dt;
  if (dgamma > 0.0) return std::min(cap, std::max(1.0, (1.0 - q.gamma0) / dgamma));
  const double g = std::fabs(q.gamma0);
  if (g >= 1.0 || q.T <= 0.0 || q.V0 <= 0.0) return cap;
  const double c = std::sqrt(1.0 - g * g);
  const double du = 2.0 * q.V0 * (c - g * std::acos(g));
  const double omega = std::sqrt(q.V0) * std::sqrt(c);
  const double expo = du / q.T;
  if (expo > 700.0) return cap;
  const double steps = 2.0 * M_PI * std::exp(expo) / (omega * q.dt);
  return std::min(cap, std::max(1.0, steps));
}

fpt_status make_plan(const fpt_params* params, int32_t n_sets, int32_t precision,
                     const fpt_tuning* tuning, Plan** out) {
  if (!params || n_sets < 1) return fail(FPT_E_INVAL, "need at least one parameter set");
  // histogram keys are (set << 12 | bin) in 32 bits with 0xFFFFFFFF as the
  // empty-slot marker: set 2^20 - 1 with bin 4095 would collide with it
  if (n_sets > kMaxPlanSets)
    return fail(FPT_E_INVAL, "at most %d parameter sets", kMaxPlanSets);
  if (precision != FPT_FP64 && precision != FPT_FP32C)
    return fail(FPT_E_INVAL, "precision %d is not FPT_FP64 or FPT_FP32C", precision);
  for (int32_t i = 0; i < n_sets; ++i) FPT_TRY(validate_params(params[i], i));
  for (int32_t i = 1; i < n_sets; ++i)
    if (integrator_kind(params[i]) != integrator_kind(params[0]))
      return fail(FPT_E_INVAL, "set %d: all sets of a plan must share one model and scheme",
                  i);
  const bool mt = params[0].rng == FPT_RNG_MT19937;
  if (mt && n_sets > 1)
    return fail(FPT_E_INVAL, "an MT19937 (rng 1) plan takes one parameter set");
  fpt_tuning t{};
  if (tuning) t = *tuning;
  if (t.schedule != FPT_SCHED_REFILL && t.schedule != FPT_SCHED_ONE_PER_LANE)
    return fail(FPT_E_INVAL, "tuning.schedule %d unknown", t.schedule);
  if (t.replicas_per_lane < 0 || t.replicas_per_lane > kMaxReplicasPerLane)
    return fail(FPT_E_INVAL, "tuning.replicas_per_lane must be 0, 1 or 2");
  if (t.waves_per_simd < 0 || t.waves_per_simd > kMaxWavesPerSimd)
    return fail(FPT_E_INVAL, "tuning.waves_per_simd must be in [0, %d]", kMaxWavesPerSimd);
  if (t.steps_per_launch < 0 || t.steps_per_launch % 4 || t.steps_per_launch > (1 << 26))
    return fail(FPT_E_INVAL, "tuning.steps_per_launch must be a multiple of 4 in [0, 2^26]");
  if (mt) {
    if (t.replicas_per_lane > 1)
      return fail(FPT_E_INVAL, "an MT19937 plan runs one replica per lane");
    t.replicas_per_lane = 1;
  }

  Plan* p = new Plan();
  p->precision = precision;
  p->model = integrator_kind(params[0]);
  p->tuning_req = t;
  p->multi = n_sets > 1;
  p->mt = mt;
  uint64_t off = 0;
  for (int32_t i = 0; i < n_sets; ++i) {
    p->params.push_back(params[i]);
    SetDev s = derive_set(params[i]);
    s.hist_off = off;
    off += s.n_bins;
    p->total_replicas += s.n_replicas;
    p->sets.push_back(s);
  }
  p->hist_bins = off;
  p->upload = p->sets;
  if (p->multi) {
    // the work queue takes the sets longest-expected first, so the replicas
    // that set the end of the run start early (results do not depend on it)
    std::vector<int32_t> order((size_t)n_sets);
    std::vector<double> est((size_t)n_sets);
    for (int32_t i = 0; i < n_sets; ++i) {
      order[(size_t)i] = i;
      est[(size_t)i] = expected_steps(params[i]);
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return est[(size_t)x] > est[(size_t)y]; });
    for (int32_t i : order) {
      const uint64_t n = (uint64_t)params[i].n_replicas;
      for (uint64_t first = 0; first < n; first += kChunk) {
        Chunk c;
        c.set = (uint32_t)i;
        c.count = (uint32_t)std::min<uint64_t>(kChunk, n - first);
        c.first = first;
        p->chunks.push_back(c);
      }
    }
    p->total_flat = (uint64_t)p->chunks.size() * kChunk;
  } else {
    p->total_flat = p->total_replicas;
  }
  p->layout();
  *out = p;
  return FPT_OK;
}

}  // namespace fpt

// ---------------------------------------------------------------------------
// C ABI

using fpt::Plan;

extern "C" {

const char* fpt_last_error(void) { return fpt::last_error(); }

int32_t fpt_api_version(void) { return FPT_API_VERSION; }

fpt_status fpt_plan(const fpt_params* sets, int32_t n_sets, int32_t precision,
                    const fpt_tuning* tuning, fpt_plan_t* out) {
  if (!out) return fpt::fail(FPT_E_INVAL, "out is NULL");
  *out = nullptr;
  Plan* p = nullptr;
  fpt_status st = fpt::make_plan(sets, n_sets, precision, tuning, &p);
  if (st != FPT_OK) return st;
  *out = new fpt_plan_s{p};
  return FPT_OK;
}

fpt_status fpt_plan_workspace(fpt_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fpt::fail(FPT_E_INVAL, "NULL argument");
  *bytes = plan->impl->ws_bytes;
  return FPT_OK;
}

fpt_status fpt_simulate(fpt_plan_t plan, void* workspace, int64_t* const* out_steps,
                        uint64_t* out_hist, void* stream) {
  if (!plan) return fpt::fail(FPT_E_INVAL, "plan is NULL");
  return plan->impl->simulate(workspace, out_steps, out_hist,
                              static_cast<hipStream_t>(stream));
}

fpt_status fpt_histogram(fpt_plan_t plan, int32_t set, uint64_t* host_counts,
                         fpt_moments* host_m) {
  if (!plan) return fpt::fail(FPT_E_INVAL, "plan is NULL");
  return plan->impl->histogram(set, host_counts, host_m);
}

fpt_status fpt_histogram_all(fpt_plan_t plan, uint64_t* host_counts, fpt_moments* host_m) {
  if (!plan) return fpt::fail(FPT_E_INVAL, "plan is NULL");
  return plan->impl->histogram_all(host_counts, host_m);
}

fpt_status fpt_plan_stats(fpt_plan_t plan, fpt_run_stats* out) {
  if (!plan || !out) return fpt::fail(FPT_E_INVAL, "NULL argument");
  return plan->impl->run_stats(out);
}

void fpt_plan_destroy(fpt_plan_t plan) {
  if (!plan) return;
  delete plan->impl;
  delete plan;
}

fpt_status fpt_rng_words(uint64_t seed, uint64_t replica0, int64_t n_rep, uint64_t block0,
                         int64_t n_blk, uint32_t* out, void* stream) {
  if (n_rep < 0 || n_blk < 0 || (n_rep * n_blk > 0 && !out))
    return fpt::fail(FPT_E_INVAL, "bad sizes or NULL output");
  FPT_HIP(fpt::launch_rng_words(seed, replica0, (uint64_t)n_rep, block0, (uint64_t)n_blk, out,
                                static_cast<hipStream_t>(stream)));
  return FPT_OK;
}

fpt_status fpt_normals(uint64_t seed, uint64_t replica0, int64_t n_rep, uint64_t block0,
                       int64_t n_blk, int32_t precision, void* out, void* stream) {
  if (n_rep < 0 || n_blk < 0 || (n_rep * n_blk > 0 && !out))
    return fpt::fail(FPT_E_INVAL, "bad sizes or NULL output");
  if (precision != FPT_FP64 && precision != FPT_FP32C)
    return fpt::fail(FPT_E_INVAL, "precision %d unknown", precision);
  FPT_HIP(fpt::launch_normals(precision == FPT_FP64, seed, replica0, (uint64_t)n_rep, block0,
                              (uint64_t)n_blk, out, static_cast<hipStream_t>(stream)));
  return FPT_OK;
}

fpt_status fpt_trajectory(const fpt_params* params, uint64_t replica, int64_t n_steps,
                          int32_t precision, double* out_phi, double* out_v, void* stream) {
  if (!params || n_steps < 0 || (n_steps > 0 && (!out_phi || !out_v)))
    return fpt::fail(FPT_E_INVAL, "bad arguments");
  if (precision != FPT_FP64 && precision != FPT_FP32C)
    return fpt::fail(FPT_E_INVAL, "precision %d unknown", precision);
  FPT_TRY(fpt::validate_params(*params, 0));
  const fpt::SetDev sd = fpt::derive_set(*params);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (params->rng != FPT_RNG_MT19937 || n_steps == 0) {
    FPT_HIP(fpt::launch_trajectory(precision == FPT_FP64, (int)sd.model, sd, replica,
                                   n_steps, out_phi, out_v, nullptr, st));
    return FPT_OK;
  }
  fpt::DeviceBuffer state;
  FPT_TRY(state.alloc(sizeof(uint4) * fpt::kMtGroupsPerSlot));
  FPT_HIP(fpt::launch_trajectory(precision == FPT_FP64, (int)sd.model, sd, replica, n_steps,
                                 out_phi, out_v, static_cast<uint4*>(state.ptr), st));
  FPT_HIP(hipStreamSynchronize(st));
  return FPT_OK;
}

fpt_status fpt_mt_words(uint64_t seed, uint64_t replica0, int64_t n_rep, uint64_t block0,
                        int64_t n_blk, uint32_t* out, void* stream) {
  if (n_rep < 0 || n_blk < 0 || (n_rep * n_blk > 0 && !out))
    return fpt::fail(FPT_E_INVAL, "bad sizes or NULL output");
  if (n_rep > (int64_t(1) << 24) || block0 > (uint64_t(1) << 24) ||
      (uint64_t)n_blk > (uint64_t(1) << 24) - block0)
    return fpt::fail(FPT_E_INVAL, "n_rep above 2^24 or blocks beyond 2^24");
  if (n_rep == 0 || n_blk == 0) return FPT_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  fpt::DeviceBuffer state;
  FPT_TRY(state.alloc(sizeof(uint4) * fpt::kMtGroupsPerSlot * (uint64_t)n_rep));
  FPT_HIP(fpt::launch_mt_words(seed, replica0, (uint64_t)n_rep, block0, (uint64_t)n_blk,
                               static_cast<uint4*>(state.ptr), out, st));
  FPT_HIP(hipStreamSynchronize(st));
  return FPT_OK;
}

}  // extern "C"
