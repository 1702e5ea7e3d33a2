// autotune.cpp -- the library's own autotuner.
//
// The integrator's results do not depend on the launch shape (every replica's
// noise is keyed by its own index), so the shape is free to tune: replicas per
// lane R (register-level ILP), resident waves per SIMD W (occupancy) and steps
// per launch S.  Candidates run a few short launches on the plan's own
// parameter sets (outputs discarded, counters reset afterwards); the shape
// with the highest measured slot-steps/s, discounted by the fill of the last
// round of replicas when they outnumber the slots, wins.  S is then sized from the
// winner's steps/s per resident slot so that one launch lasts about
// FPT_LAUNCH_MS milliseconds (default 40); FPT_TUNE_VERBOSE=1 prints each
// trial.  Winners are
// cached in memory and in a JSON-lines file (FPT_TUNE_CACHE, default
// $HOME/.cache/fpt_tune.jsonl), one object per key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "autotune.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace fpt {

namespace {
std::mutex g_mu;
std::map<std::string, TuneEntry> g_cache;
bool g_loaded = false;

std::string cache_path() {
  if (const char* p = std::getenv("FPT_TUNE_CACHE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/fpt_tune.jsonl";
}

void load_file_locked() {
  if (g_loaded) return;
  g_loaded = true;
  FILE* f = std::fopen(cache_path().c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char key[256];
    TuneEntry e;
    if (std::sscanf(line,
                    "{\"key\": \"%255[^\"]\", \"R\": %d, \"W\": %d, \"rate\": %lf, "
                    "\"slot_rate\": %lf}",
                    key, &e.replicas_per_lane, &e.waves_per_simd, &e.slot_steps_per_s,
                    &e.per_slot_steps_per_s) == 5)
      g_cache[key] = e;
  }
  std::fclose(f);
}

double launch_ms_target() {
  if (const char* p = std::getenv("FPT_LAUNCH_MS")) {
    const double v = std::atof(p);
    if (v > 0) return v;
  }
  return 40.0;
}
}  // namespace

// FPT_TUNE_VERBOSE=1 prints every trial to stderr.
static bool tune_verbose() {
  const char* v = std::getenv("FPT_TUNE_VERBOSE");
  return v && v[0] == '1';
}

// Entries are kept per build of the library (its kernels may change the best
// shape), per device, precision, model, schedule and single / multi set.
std::string tune_key(const std::string& arch, int precision, int model, int schedule,
                     bool multi) {
  static const char kBuild[] = __DATE__ " " __TIME__;
  char buf[200];
  std::snprintf(buf, sizeof(buf), "%s/%s/p%d/m%d/s%d/%s", kBuild, arch.c_str(), precision,
                model, schedule, multi ? "multi" : "single");
  return buf;
}

bool tune_lookup(const std::string& key, TuneEntry* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

void tune_store(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  g_cache[key] = e;
  const std::string path = cache_path();
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;  // the cache file is an optimisation only
  std::fprintf(f,
               "{\"key\": \"%s\", \"R\": %d, \"W\": %d, \"rate\": %.6e, \"slot_rate\": %.6e}\n",
               key.c_str(), e.replicas_per_lane, e.waves_per_simd, e.slot_steps_per_s,
               e.per_slot_steps_per_s);
  std::fclose(f);
}

// Measure one candidate shape: a warm-up launch of 256 blocks (1024 steps)
// whose duration sizes the two timed launches to about 8 ms each, so launch
// overhead and the ramp-up of the persistent grid do not decide the ranking.
// Returns slot-steps/s (negative if the shape does not fit the workspace).
static fpt_status trial(Plan& p, char* ws, hipStream_t st, const fpt_tuning& t,
                        double* rate, double* slot_rate) {
  const int R = t.replicas_per_lane;
  const bool refill = t.schedule == FPT_SCHED_REFILL;
  const uint64_t lanes = p.lanes_for(t);
  *slot_rate = 0.0;
  if (lanes * (uint64_t)R > p.max_slots) {
    *rate = -1.0;
    return FPT_OK;
  }
  std::vector<SetDev> table = p.sets;
  for (SetDev& s : table) s.out_steps = nullptr;
  FPT_TRY(p.upload_sets(ws, table, st));
  uint64_t* hist = reinterpret_cast<uint64_t*>(ws + p.off_hist);
  SliceArgs a = p.slice_args(ws, hist, lanes);
  a.blocks = 256;
  a.refill = refill ? 1 : 0;
  a.whole_waves = p.regroups(t) ? 1 : 0;
  FPT_TRY(p.reset_run(ws, a, lanes, R, refill, st));
  FPT_TRY(p.ensure_host_resources(3));
  const uint32_t groups = (uint32_t)(lanes / kBlockThreads);
  const bool fp64 = p.precision == FPT_FP64;
  FPT_HIP(hipEventRecord(p.events[0], st));
  FPT_HIP(launch_slice(fp64, p.model, R, p.multi, a, groups, st));
  FPT_HIP(hipEventRecord(p.events[1], st));
  FPT_HIP(hipStreamSynchronize(st));
  float warm_ms = 0.f;
  FPT_HIP(hipEventElapsedTime(&warm_ms, p.events[0], p.events[1]));
  const double scale = warm_ms > 0.f ? 8.0 / (double)warm_ms : 1.0;
  a.blocks = (int32_t)std::max(256.0, std::min(256.0 * scale, 262144.0));
  FPT_HIP(hipMemcpyAsync(p.h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  FPT_HIP(hipStreamSynchronize(st));
  const unsigned long long before = p.h_ctr->lane_steps;
  FPT_HIP(hipEventRecord(p.events[0], st));
  for (int i = 0; i < 2; ++i)
    FPT_HIP(launch_slice(fp64, p.model, R, p.multi, a, groups, st));
  FPT_HIP(hipEventRecord(p.events[1], st));
  FPT_HIP(hipMemcpyAsync(p.h_ctr, a.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  FPT_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  FPT_HIP(hipEventElapsedTime(&ms, p.events[0], p.events[1]));
  const double steps = (double)(p.h_ctr->lane_steps - before);
  *rate = ms > 0.f ? steps / (ms * 1e-3) : 0.0;
  *slot_rate = *rate / (double)(lanes * (uint64_t)R);
  return FPT_OK;
}

// Resident waves per SIMD of the plan's kernel with R replicas per lane
// (kMaxWavesPerSimd if the runtime cannot say).
int Plan::resident_waves(int R) const {
  const int n = slice_resident_groups(precision == FPT_FP64, model, R, multi, mt);
  return n > 0 ? std::min(n, kMaxWavesPerSimd) : kMaxWavesPerSimd;
}

fpt_status Plan::resolve_tuning(char* ws, hipStream_t st) {
  fpt_tuning t = tuning_req;
  const bool need_r = t.replicas_per_lane == 0;
  const bool need_w = t.waves_per_simd == 0;
  const bool need_s = t.steps_per_launch == 0;
  TuneEntry best;
  bool have_rate = false;
  if (need_r || need_w || need_s) {
    // the size class matters: below the chip's lane capacity every wave
    // count gives the same lane count, so a small plan's winner says nothing
    // about a large one
    int size_class = 0;
    for (uint64_t n = total_flat; n > 1; n >>= 1) ++size_class;
    const std::string key = tune_key(arch, precision, model, t.schedule, multi) + "/n" +
                            std::to_string(size_class) + (mt ? "/mt19937" : "");
    TuneEntry cached;
    if (tune_lookup(key, &cached)) {
      if (need_r) t.replicas_per_lane = cached.replicas_per_lane;
      if (need_w) t.waves_per_simd = cached.waves_per_simd;
      best = cached;
      have_rate = cached.per_slot_steps_per_s > 0;
    } else if (total_replicas > 0) {
      std::vector<int> rs = need_r ? std::vector<int>{1, 2}
                                   : std::vector<int>{t.replicas_per_lane};
      double best_rate = -1.0;
      for (int r : rs) {
        // every resident wave count from 2 up to the kernel's occupancy:
        // more would leave workgroups of the persistent grid waiting
        const int occ = resident_waves(r);
        std::vector<int> ws_list;
        if (!need_w) {
          ws_list = {std::min(t.waves_per_simd, occ)};
        } else if (t.schedule == FPT_SCHED_ONE_PER_LANE) {
          ws_list = {occ};
        } else {
          for (int w = std::min(2, occ); w <= occ; ++w) ws_list.push_back(w);
        }
        for (int w : ws_list) {
          fpt_tuning c = t;
          c.replicas_per_lane = r;
          c.waves_per_simd = w;
          double rate = 0.0, slot_rate = 0.0;
          FPT_TRY(trial(*this, ws, st, c, &rate, &slot_rate));
          // replicas of similar lifetime run in rounds of one per slot; a
          // last round that fills only part of the slots idles the rest, so
          // the shape is ranked by its rate times that round's fill
          const double slots = (double)(lanes_for(c) * (uint64_t)r);
          const double rounds = slots > 0 ? (double)total_flat / slots : 1.0;
          const double fill = rounds <= 1.0 ? 1.0 : rounds / std::ceil(rounds);
          const double score = rate * fill;
          if (tune_verbose())
            std::fprintf(stderr,
                         "[fpt tune] R=%d W=%d lanes=%llu rate=%.4e slot-steps/s fill=%.3f "
                         "score=%.4e\n",
                         r, w, (unsigned long long)lanes_for(c), rate, fill, score);
          if (score > best_rate) {
            best_rate = score;
            best.replicas_per_lane = r;
            best.waves_per_simd = w;
            best.slot_steps_per_s = rate;
            best.per_slot_steps_per_s = slot_rate;
          }
        }
      }
      if (best_rate > 0) {
        t.replicas_per_lane = best.replicas_per_lane;
        t.waves_per_simd = best.waves_per_simd;
        have_rate = true;
        tune_store(key, best);
      }
    }
  }
  if (t.replicas_per_lane == 0) t.replicas_per_lane = 1;
  if (t.waves_per_simd == 0) t.waves_per_simd = kMaxWavesPerSimd;
  t.waves_per_simd = std::min(t.waves_per_simd, resident_waves(t.replicas_per_lane));
  if (need_s) {
    uint64_t s = 16384;
    if (have_rate && best.per_slot_steps_per_s > 0)
      s = (uint64_t)(launch_ms_target() * 1e-3 * best.per_slot_steps_per_s);
    s = std::max<uint64_t>(256, std::min<uint64_t>(s, uint64_t(1) << 20));
    t.steps_per_launch = (int32_t)(s / 4 * 4);
  }
  tuning = t;
  return FPT_OK;
}

}  // namespace fpt
