// server.cpp -- continuous batching of first-passage-time jobs.
//
// The paper's host loop hands a new realization to a processor as soon as
// the previous one ends (Sect. III.B, the streaming figure).  Here that loop
// runs at two levels: on the device, persistent lanes draw replicas from a
// ring of work chunks (kernels.hip); on the host, a request thread admits
// whole jobs into the ring between launches as set slots, histogram memory
// and ring space free up, and retires jobs whose replicas have all finished.
// Lane state stays resident in the caller's pool across launches, so jobs
// that arrive while others run share the same launches.
//
// Pool layout (caller-owned device memory):
//   set table [max_sets] | chunk ring [ring] | counters | moments [max_sets]
//   | lane state [slots] | histogram region (first-fit allocated per job)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "autotune.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace fpt {

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxSets = 1024;
constexpr uint64_t kMinRingChunks = 1 << 12;
constexpr uint64_t kMaxRingChunks = 1 << 22;
constexpr size_t kMaxQueued = 1 << 20;

enum class JobState { Queued, Running, Done };

struct Job {
  uint64_t id = 0;
  fpt_params params{};
  SetDev dev{};
  JobState state = JobState::Queued;
  int32_t slot = -1;
  uint64_t hist_off = 0;       // in the histogram region, uint64 units
  uint64_t n_chunks = 0;
  Clock::time_point t_submit, t_done;
  std::vector<uint64_t> counts;
  fpt_moments mom{};
};

// First-fit allocator of [0, capacity) in uint64 units.
class RangeAlloc {
 public:
  explicit RangeAlloc(uint64_t cap = 0) { if (cap) free_[0] = cap; cap_ = cap; }
  bool alloc(uint64_t n, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t capacity() const { return cap_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t cap_ = 0;
};

}  // namespace

struct Server {
  char* pool = nullptr;
  size_t pool_bytes = 0;
  int precision = FPT_FP32C;
  int model = FPT_UNDERDAMPED;
  fpt_tuning tuning{};
  hipStream_t stream = nullptr;
  int device = 0;

  uint64_t n_lanes = 0, n_slots = 0, ring = 0;
  uint64_t off_sets = 0, off_chunks = 0, off_ctr = 0, off_mom = 0;
  uint64_t off_st_phi = 0, off_st_v = 0, off_st_j = 0, off_st_idx = 0, off_st_set = 0;
  // second lane-state buffer: when the ring is drained the active slots are
  // compacted into a prefix of the other buffer and launches narrow to
  // cur_lanes; appended work widens them again (the slots past the prefix
  // are marked free in the whole buffer)
  uint64_t off_alt[5] = {0, 0, 0, 0, 0};
  int buf = 0;
  uint64_t cur_lanes = 0;
  uint64_t off_group = 0;      // per-set positions of a move in set order
  uint64_t off_hist = 0;
  RangeAlloc hist_alloc;

  Counters* h_ctr = nullptr;   // pinned
  MomDev* h_mom = nullptr;     // pinned, kMaxSets

  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::string thread_error;
  std::deque<Job*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  std::vector<Job*> slot_job = std::vector<Job*>(kMaxSets, nullptr);
  uint64_t next_id = 1;
  uint64_t chunk_tail = 0;     // chunks appended so far
  uint64_t cursor_seen = 0;    // device cursor at the last sync
  fpt_server_stats stats{};
  Clock::time_point busy_since;
  bool busy = false;
  std::thread th;

  SliceArgs args() const { return args_for(buf, cur_lanes); }

  SliceArgs args_for(int b, uint64_t lanes) const {
    SliceArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sets = reinterpret_cast<const SetDev*>(pool + off_sets);
    a.chunks = reinterpret_cast<const Chunk*>(pool + off_chunks);
    a.chunk_mask = ring - 1;
    a.ctr = reinterpret_cast<Counters*>(pool + off_ctr);
    a.total = chunk_tail * kChunk;
    const uint64_t o_phi = b ? off_alt[0] : off_st_phi, o_v = b ? off_alt[1] : off_st_v,
                   o_j = b ? off_alt[2] : off_st_j, o_idx = b ? off_alt[3] : off_st_idx,
                   o_set = b ? off_alt[4] : off_st_set;
    a.st_phi = reinterpret_cast<unsigned long long*>(pool + o_phi);
    a.st_v = reinterpret_cast<unsigned long long*>(pool + o_v);
    a.st_j = reinterpret_cast<unsigned long long*>(pool + o_j);
    a.st_idx = reinterpret_cast<unsigned long long*>(pool + o_idx);
    a.st_set = reinterpret_cast<uint32_t*>(pool + o_set);
    a.n_lanes = lanes;
    a.hist = reinterpret_cast<unsigned long long*>(pool + off_hist);
    a.mom = reinterpret_cast<MomDev*>(pool + off_mom);
    a.blocks = tuning.steps_per_launch / 4;
    a.refill = 1;
    a.clamp = 1;
    a.whole_waves = tuning.no_regroup ? 0 : 1;
    return a;
  }

  fpt_status setup();
  void loop();
  fpt_status admit_locked(Job* j);
  fpt_status step();
  fpt_status maybe_compact_locked();
  void finish_locked(Job* j, const MomDev& m);
};

fpt_status Server::setup() {
  const DeviceInfo di = device_info();
  device = di.device;
  if (tuning.replicas_per_lane == 0 || tuning.waves_per_simd == 0) {
    TuneEntry e;
    if (tune_lookup(tune_key(di.arch, precision, model, FPT_SCHED_REFILL, true), &e)) {
      if (!tuning.replicas_per_lane) tuning.replicas_per_lane = e.replicas_per_lane;
      if (!tuning.waves_per_simd) tuning.waves_per_simd = e.waves_per_simd;
    }
  }
  if (!tuning.replicas_per_lane) tuning.replicas_per_lane = 1;
  if (!tuning.waves_per_simd) tuning.waves_per_simd = kMaxWavesPerSimd;
  {
    // no more persistent workgroups than fit on the chip at once
    const int occ = slice_resident_groups(precision == FPT_FP64, model,
                                          tuning.replicas_per_lane, true, false);
    if (occ > 0) tuning.waves_per_simd = std::min(tuning.waves_per_simd, occ);
  }
  if (!tuning.steps_per_launch) tuning.steps_per_launch = 8192;
  tuning.schedule = FPT_SCHED_REFILL;
  n_lanes = (uint64_t)di.cus * 4 * (uint64_t)tuning.waves_per_simd * kWave;
  n_slots = n_lanes * (uint64_t)tuning.replicas_per_lane;

  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  off_sets = take(sizeof(SetDev) * kMaxSets);
  off_ctr = take(sizeof(Counters));
  off_mom = take(sizeof(MomDev) * kMaxSets);
  off_st_phi = take(8 * n_slots);
  off_st_v = take(8 * n_slots);
  off_st_j = take(8 * n_slots);
  off_st_idx = take(8 * n_slots);
  off_st_set = take(4 * n_slots);
  off_alt[0] = take(8 * n_slots);
  off_alt[1] = take(8 * n_slots);
  off_alt[2] = take(8 * n_slots);
  off_alt[3] = take(8 * n_slots);
  off_alt[4] = take(4 * n_slots);
  off_group = take(2 * sizeof(unsigned long long) * kMaxSets);  // counts, first positions
  cur_lanes = n_lanes;
  if (off + sizeof(Chunk) * kMinRingChunks + 8 * FPT_MAX_BINS > pool_bytes)
    return fail(FPT_E_NOMEM, "pool of %zu bytes cannot hold the lane state (%llu bytes) "
                "plus a minimal work ring and one histogram", pool_bytes,
                (unsigned long long)off);
  // half of the rest (at most 4M chunks) for the ring, the rest for histograms
  const uint64_t rest = pool_bytes - off;
  ring = kMinRingChunks;
  while (ring * 2 <= kMaxRingChunks && sizeof(Chunk) * ring * 2 <= rest / 2) ring *= 2;
  off_chunks = take(sizeof(Chunk) * ring);
  off_hist = off;
  hist_alloc = RangeAlloc((pool_bytes - off_hist) / 8);

  FPT_HIP(hipSetDevice(device));
  FPT_HIP(hipHostMalloc((void**)&h_ctr, sizeof(Counters), hipHostMallocDefault));
  FPT_HIP(hipHostMalloc((void**)&h_mom, sizeof(MomDev) * kMaxSets, hipHostMallocDefault));
  const SliceArgs a = args();
  FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(a.ctr), sizeof(Counters) / 8,
                          0ull, stream));
  FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(a.mom),
                          sizeof(MomDev) / 8 * kMaxSets, 0ull, stream));
  FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(pool + off_group), kMaxSets,
                          0ull, stream));
  FPT_HIP(launch_init(precision == FPT_FP64, a, n_slots, 0, stream));
  FPT_HIP(hipStreamSynchronize(stream));
  return FPT_OK;
}

// Admission: a free set slot, histogram memory and ring space.
fpt_status Server::admit_locked(Job* j) {
  int32_t slot = -1;
  for (int32_t i = 0; i < kMaxSets; ++i)
    if (!slot_job[(size_t)i]) {
      slot = i;
      break;
    }
  if (slot < 0) return FPT_E_BUSY;
  const uint64_t cursor_chunks = cursor_seen / kChunk;
  if (chunk_tail + j->n_chunks - cursor_chunks > ring) return FPT_E_BUSY;
  uint64_t hoff = 0;
  if (!hist_alloc.alloc((uint64_t)j->params.n_bins, &hoff)) return FPT_E_BUSY;

  j->slot = slot;
  j->hist_off = hoff;
  SetDev d = j->dev;
  d.hist_off = hoff;
  d.out_steps = nullptr;
  const SliceArgs a = args();
  FPT_HIP(hipMemcpyAsync(pool + off_sets + sizeof(SetDev) * (size_t)slot, &d, sizeof(SetDev),
                         hipMemcpyHostToDevice, stream));
  FPT_HIP(launch_fill_u64(a.hist + hoff, (uint64_t)j->params.n_bins, 0ull, stream));
  FPT_HIP(launch_fill_u64(reinterpret_cast<unsigned long long*>(a.mom + slot),
                          sizeof(MomDev) / 8, 0ull, stream));
  std::vector<Chunk> ch(j->n_chunks);
  const uint64_t n = (uint64_t)j->params.n_replicas;
  for (uint64_t c = 0; c < j->n_chunks; ++c) {
    ch[c].set = (uint32_t)slot;
    ch[c].first = c * kChunk;
    ch[c].count = (uint32_t)std::min<uint64_t>(kChunk, n - c * kChunk);
  }
  uint64_t done = 0;
  while (done < j->n_chunks) {
    const uint64_t pos = (chunk_tail + done) & (ring - 1);
    const uint64_t len = std::min(j->n_chunks - done, ring - pos);
    FPT_HIP(hipMemcpyAsync(pool + off_chunks + sizeof(Chunk) * pos, ch.data() + done,
                           sizeof(Chunk) * len, hipMemcpyHostToDevice, stream));
    done += len;
  }
  // pageable sources: make the copies complete before `ch` goes away
  FPT_HIP(hipStreamSynchronize(stream));
  chunk_tail += j->n_chunks;
  cur_lanes = n_lanes;  // new work: full width again
  slot_job[(size_t)slot] = j;
  j->state = JobState::Running;
  ++stats.admitted;
  ++stats.running;
  --stats.queued;
  if (n == 0) {
    MomDev zero{};
    finish_locked(j, zero);
  }
  return FPT_OK;
}

void Server::finish_locked(Job* j, const MomDev& m) {
  j->counts.assign((size_t)j->params.n_bins, 0);
  if (j->params.n_bins > 0 && j->params.n_replicas > 0) {
    if (hipMemcpyAsync(j->counts.data(), pool + off_hist + 8 * j->hist_off,
                       8 * (size_t)j->params.n_bins, hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      // the device is in doubt: stop the loop (pending polls report it)
      thread_error = "histogram readback failed";
      stop = true;
    }
  }
  fill_moments(m, j->params.dt, &j->mom);
  hist_alloc.release(j->hist_off, (uint64_t)j->params.n_bins);
  slot_job[(size_t)j->slot] = nullptr;
  j->state = JobState::Done;
  j->t_done = Clock::now();
  ++stats.finished;
  --stats.running;
  stats.replica_steps += m.sum_k + m.n_cens * (uint64_t)j->params.max_steps;
}

// One launch over all admitted work, then retire finished jobs.
fpt_status Server::step() {
  SliceArgs a;
  int buf_seen = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    a = args();
    buf_seen = buf;
  }
  const uint32_t groups = (uint32_t)(a.n_lanes / kBlockThreads);
  FPT_HIP(launch_slice(precision == FPT_FP64, model, tuning.replicas_per_lane, true, a, groups,
                       stream));
  if (a.whole_waves && cursor_seen < a.total) {
    // the active slots into set order, the free ones past them refilled in
    // queue order (lanes of a wavefront share a set again)
    const uint64_t slots = a.n_lanes * (uint64_t)tuning.replicas_per_lane;
    const SliceArgs other = args_for(1 - buf_seen, a.n_lanes);
    auto* counts = reinterpret_cast<unsigned long long*>(pool + off_group);
    auto* first = counts + kMaxSets;
    FPT_HIP(launch_group_count(a, slots, counts, first, kMaxSets, stream));
    FPT_HIP(launch_group_move(a, other, slots, slots, first, stream));
    FPT_HIP(launch_group_refill(precision == FPT_FP64, other, slots, stream));
    FPT_HIP(launch_copy_state(other, a, slots, true, stream));
    ++stats.n_regroups;
  }
  FPT_HIP(hipMemcpyAsync(h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
  FPT_HIP(hipMemcpyAsync(h_mom, a.mom, sizeof(MomDev) * kMaxSets, hipMemcpyDeviceToHost,
                         stream));
  FPT_HIP(hipStreamSynchronize(stream));
  std::lock_guard<std::mutex> lk(mu);
  ++stats.n_launches;
  if (h_ctr->overflow) return fail(FPT_E_DEVICE, "regroup could not place slots");
  cursor_seen = h_ctr->cursor;
  for (int32_t i = 0; i < kMaxSets; ++i) {
    Job* j = slot_job[(size_t)i];
    if (!j) continue;
    const MomDev& m = h_mom[i];
    if (m.n_esc + m.n_cens >= (uint64_t)j->params.n_replicas) finish_locked(j, m);
  }
  if (stats.running > 0) FPT_TRY(maybe_compact_locked());
  return FPT_OK;
}

// With every appended replica drawn and the active ones filling at most 80%
// of the current slots, move them in set order to a dense prefix of the other
// lane-state buffer (whose remaining slots, up to the full width, are marked
// free) and narrow the launches; admit_locked widens them again.
fpt_status Server::maybe_compact_locked() {
  const uint64_t total = chunk_tail * kChunk;
  if (h_ctr->cursor < total || cur_lanes <= (uint64_t)kBlockThreads) return FPT_OK;
  const uint64_t R = (uint64_t)tuning.replicas_per_lane;
  const uint64_t slots = cur_lanes * R;
  const uint64_t active_bound = h_ctr->cursor - std::min<uint64_t>(h_ctr->cursor, h_ctr->done);
  if (active_bound * 10 > slots * 8) return FPT_OK;
  const SliceArgs a = args();
  auto* counts = reinterpret_cast<unsigned long long*>(pool + off_group);
  auto* first = counts + kMaxSets;
  FPT_HIP(launch_group_count(a, slots, counts, first, kMaxSets, stream));
  FPT_HIP(hipMemcpyAsync(h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
  FPT_HIP(hipStreamSynchronize(stream));
  const uint64_t active = h_ctr->compact;
  const uint64_t lanes =
      std::max<uint64_t>(kBlockThreads, round_up((active + R - 1) / R, kBlockThreads));
  if (lanes * 10 > cur_lanes * 9) return FPT_OK;
  SliceArgs dst = args_for(1 - buf, lanes);
  FPT_HIP(launch_group_move(a, dst, slots, n_slots, first, stream));
  FPT_HIP(hipStreamSynchronize(stream));
  buf = 1 - buf;
  cur_lanes = lanes;
  ++stats.n_compactions;
  return FPT_OK;
}

void Server::loop() {
  if (hipSetDevice(device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    thread_error = "hipSetDevice failed in the server thread";
    stop = true;
    return;
  }
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        while (!queue.empty()) {
          const fpt_status st = admit_locked(queue.front());
          if (st == FPT_E_BUSY) break;
          if (st != FPT_OK) {
            thread_error = last_error();
            stop = true;
            break;
          }
          queue.pop_front();
        }
        if (stop) return;
        if (stats.running > 0) break;
        if (busy) {
          stats.busy_s += std::chrono::duration<double>(Clock::now() - busy_since).count();
          busy = false;
        }
        cv.wait(lk);
      }
      if (!busy) {
        busy = true;
        busy_since = Clock::now();
      }
    }
    if (step() != FPT_OK) {
      std::lock_guard<std::mutex> lk(mu);
      thread_error = last_error();
      stop = true;
      return;
    }
  }
}

}  // namespace fpt

// ---------------------------------------------------------------------------
// C ABI

struct fpt_server_s {
  fpt::Server* impl;
};

extern "C" {

fpt_status fpt_server_create(void* device_pool, size_t pool_bytes, int32_t precision,
                             int32_t model, int32_t scheme, const fpt_tuning* tuning,
                             void* stream, fpt_server_t* out) {
  if (!out) return fpt::fail(FPT_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!device_pool) return fpt::fail(FPT_E_INVAL, "device_pool is NULL");
  if (reinterpret_cast<uintptr_t>(device_pool) % 256)
    return fpt::fail(FPT_E_INVAL, "device_pool must be 256-byte aligned");
  if (precision != FPT_FP64 && precision != FPT_FP32C)
    return fpt::fail(FPT_E_INVAL, "precision %d unknown", precision);
  if (model != FPT_UNDERDAMPED && model != FPT_OVERDAMPED)
    return fpt::fail(FPT_E_INVAL, "model %d unknown", model);
  if (scheme != FPT_EXPLICIT && scheme != FPT_SEMI_IMPLICIT)
    return fpt::fail(FPT_E_INVAL, "scheme %d unknown", scheme);
  if (model == FPT_OVERDAMPED && scheme != FPT_EXPLICIT)
    return fpt::fail(FPT_E_INVAL, "the overdamped model has only scheme 0");
  fpt_params kind{};
  kind.model = model;
  kind.scheme = scheme;
  auto* s = new fpt::Server();
  s->pool = static_cast<char*>(device_pool);
  s->pool_bytes = pool_bytes;
  s->precision = precision;
  s->model = fpt::integrator_kind(kind);  // the one integrator every launch runs
  if (tuning) s->tuning = *tuning;
  if (s->tuning.steps_per_launch < 0 || s->tuning.steps_per_launch % 4 ||
      s->tuning.replicas_per_lane < 0 || s->tuning.replicas_per_lane > 2 ||
      s->tuning.waves_per_simd < 0 || s->tuning.waves_per_simd > fpt::kMaxWavesPerSimd) {
    delete s;
    return fpt::fail(FPT_E_INVAL, "bad tuning");
  }
  s->stream = static_cast<hipStream_t>(stream);
  const fpt_status st = s->setup();
  if (st != FPT_OK) {
    if (s->h_ctr) (void)hipHostFree(s->h_ctr);
    if (s->h_mom) (void)hipHostFree(s->h_mom);
    delete s;
    return st;
  }
  s->th = std::thread([s] { s->loop(); });
  *out = new fpt_server_s{s};
  return FPT_OK;
}

fpt_status fpt_submit(fpt_server_t server, const fpt_params* params, uint64_t* job_id) {
  if (!server || !params || !job_id) return fpt::fail(FPT_E_INVAL, "NULL argument");
  fpt::Server* s = server->impl;
  FPT_TRY(fpt::validate_params(*params, 0));
  if (params->rng != FPT_RNG_PHILOX)
    return fpt::fail(FPT_E_INVAL, "the server runs Philox jobs only (rng 0)");
  if (fpt::integrator_kind(*params) != s->model)
    return fpt::fail(FPT_E_INVAL, "job model %d / scheme %d: this server runs another "
                     "model or scheme", params->model, params->scheme);
  const uint64_t n_chunks =
      ((uint64_t)params->n_replicas + fpt::kChunk - 1) / (uint64_t)fpt::kChunk;
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->thread_error.empty())
    return fpt::fail(FPT_E_DEVICE, "server stopped: %s", s->thread_error.c_str());
  if (n_chunks > s->ring || (uint64_t)params->n_bins > s->hist_alloc.capacity())
    return fpt::fail(FPT_E_NOMEM, "job needs %llu work chunks and %d bins; the pool holds %llu "
                     "chunks and %llu bins", (unsigned long long)n_chunks, params->n_bins,
                     (unsigned long long)s->ring,
                     (unsigned long long)s->hist_alloc.capacity());
  if (s->queue.size() >= fpt::kMaxQueued) return fpt::fail(FPT_E_BUSY, "queue full");
  auto j = std::make_unique<fpt::Job>();
  j->id = s->next_id++;
  j->params = *params;
  j->dev = fpt::derive_set(*params);
  j->n_chunks = n_chunks;
  j->t_submit = fpt::Clock::now();
  *job_id = j->id;
  s->queue.push_back(j.get());
  s->jobs[j->id] = std::move(j);
  ++s->stats.submitted;
  ++s->stats.queued;
  s->cv.notify_all();
  return FPT_OK;
}

fpt_status fpt_poll(fpt_server_t server, uint64_t job_id, uint64_t* host_counts,
                    fpt_moments* host_m, double* latency_s) {
  if (!server) return fpt::fail(FPT_E_INVAL, "server is NULL");
  fpt::Server* s = server->impl;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fpt::fail(FPT_E_NOTFOUND, "job %llu unknown",
                                            (unsigned long long)job_id);
  fpt::Job* j = it->second.get();
  if (j->state != fpt::JobState::Done) {
    if (!s->thread_error.empty())
      return fpt::fail(FPT_E_DEVICE, "server stopped: %s", s->thread_error.c_str());
    return FPT_PENDING;
  }
  if (host_counts) std::copy(j->counts.begin(), j->counts.end(), host_counts);
  if (host_m) *host_m = j->mom;
  if (latency_s) *latency_s = std::chrono::duration<double>(j->t_done - j->t_submit).count();
  s->jobs.erase(it);
  return FPT_OK;
}

fpt_status fpt_server_stats_get(fpt_server_t server, fpt_server_stats* out) {
  if (!server || !out) return fpt::fail(FPT_E_INVAL, "NULL argument");
  fpt::Server* s = server->impl;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  if (s->busy)
    out->busy_s += std::chrono::duration<double>(fpt::Clock::now() - s->busy_since).count();
  return FPT_OK;
}

void fpt_server_destroy(fpt_server_t server) {
  if (!server) return;
  fpt::Server* s = server->impl;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  (void)hipStreamSynchronize(s->stream);
  if (s->h_ctr) (void)hipHostFree(s->h_ctr);
  if (s->h_mom) (void)hipHostFree(s->h_mom);
  delete s;
  delete server;
}

}  // extern "C"
