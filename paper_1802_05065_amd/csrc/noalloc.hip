// noalloc.hip -- fpt_simulate_noalloc: fpt_simulate with the workspace in a
// static device array of the library, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The array lives in the library's code object: each GPU the library runs on
// holds its own copy, at its own address, from the first use until the
// process ends.  Host code never passes the array's name to a kernel (in host
// code that name is only a stand-in, not a device address): on the first
// call on a device, with that device current, hipGetSymbolAddress gives the
// device address, which is kept per device and used from then on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.hpp"

namespace {

// Largest workspace of an allocation-free run (FPT_NOALLOC_SCRATCH_BYTES,
// 48 MiB): the lane state of 2^19 slots (8 waves per SIMD on 256 CUs, one
// replica per lane) with the compaction buffer, plus the set table, work
// queue, counters, moments and histograms of a plan of a few hundred sets.
constexpr uint64_t kScratchBytes = FPT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, resolved once
// per device.
fpt_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fpt::fail(FPT_E_DEVICE, "hipGetDevice failed");
  }
  if (dev < 0 || dev >= kMaxDevices)
    return fpt::fail(FPT_E_DEVICE, "device %d outside the %d the library tracks", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fpt::fail(FPT_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                       hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FPT_OK;
}

}  // namespace

extern "C" {

fpt_status fpt_simulate_noalloc(fpt_plan_t plan, int64_t* const* out_steps, uint64_t* out_hist,
                                void* stream) {
  if (!plan) return fpt::fail(FPT_E_INVAL, "plan is NULL");
  void* ws = nullptr;
  FPT_TRY(scratch_for_current_device(&ws));
  return plan->impl->simulate_in_scratch(ws, kScratchBytes, out_steps, out_hist,
                                         static_cast<hipStream_t>(stream));
}

}  // extern "C"
