// common.hpp -- host-side helpers of the first-passage-time runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>

#include "fpt.h"
#include "internal.hpp"

namespace fpt {

// Thread-local error text behind fpt_last_error(); returns `st`.
fpt_status fail(fpt_status st, const char* fmt, ...)
    __attribute__((format(printf, 2, 3)));
void clear_error();

#define FPT_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::fpt::fail(FPT_E_DEVICE, "%s failed: %s", #call,               \
                         hipGetErrorString(e_));                             \
  } while (0)

#define FPT_TRY(expr)                   \
  do {                                  \
    fpt_status s_ = (expr);             \
    if (s_ != FPT_OK) return s_;        \
  } while (0)

// Argument checks of one parameter set; `index` names it in the message.
fpt_status validate_params(const fpt_params& p, int index);

// Algorithm 1 / 3 preamble for one set (host, FP64).
SetDev derive_set(const fpt_params& p);

struct DeviceInfo {
  int device = 0;
  int cus = 256;
  std::string arch = "gfx950";
};
DeviceInfo device_info();

// Largest launch shape the runtime uses (sizes the workspace).
constexpr int kMaxWavesPerSimd = 8;
constexpr int kMaxReplicasPerLane = 2;

inline uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

// 16-byte groups of one slot's MT19937 state (624 words).
constexpr uint64_t kMtGroupsPerSlot = 156;

// Temporary device memory of a diagnostic call, freed on scope exit.
struct DeviceBuffer {
  void* ptr = nullptr;
  DeviceBuffer() = default;
  DeviceBuffer(const DeviceBuffer&) = delete;
  DeviceBuffer& operator=(const DeviceBuffer&) = delete;
  ~DeviceBuffer() {
    if (ptr) (void)hipFree(ptr);
  }
  fpt_status alloc(size_t bytes) {
    const hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
      ptr = nullptr;
      return fail(FPT_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return FPT_OK;
  }
};

}  // namespace fpt
