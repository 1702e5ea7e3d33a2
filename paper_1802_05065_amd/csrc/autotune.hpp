// autotune.hpp -- launch-shape tuning cache.
#pragma once

#include <string>

#include "fpt.h"

namespace fpt {

struct TuneEntry {
  int replicas_per_lane = 1;
  int waves_per_simd = 8;
  double slot_steps_per_s = 0.0;  // measured issue rate of the winning shape
  double per_slot_steps_per_s = 0.0;  // the same per resident slot
};

// Key: GPU architecture, precision, model, schedule and set-count bucket.
std::string tune_key(const std::string& arch, int precision, int model, int schedule,
                     bool multi);
bool tune_lookup(const std::string& key, TuneEntry* out);
void tune_store(const std::string& key, const TuneEntry& e);

}  // namespace fpt
