// PM force with the library's scratch in a fixed device array, for callers
// that cannot allocate device memory (tight serving loops, harnesses that
// forbid allocation).  The call waits for its table upload, so it is not
// for code under stream capture.
//
// The array below is the workspace pm_create would otherwise take from the
// caller.  Each GPU the library runs on holds its own copy for the lifetime
// of the process.  Host code never passes the array's name to a kernel or a
// copy (in host code that name is a host-side stand-in, not a device
// address): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is kept per device.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "pm.h"

namespace {

constexpr size_t kScratchBytes = (size_t)PM_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of the workspace alignment");

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_dev_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    std::fprintf(stderr, "pm_force_static: hipGetDevice: %s\n", hipGetErrorString(e));
    return PM_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    std::fprintf(stderr, "pm_force_static: device ordinal %d outside [0, %d)\n", dev, kMaxDevices);
    return PM_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_dev_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      std::fprintf(stderr, "pm_force_static: hipGetSymbolAddress on device %d: %s\n", dev,
                   hipGetErrorString(e));
      return PM_EHIP;
    }
    g_dev_ptr[dev] = p;
  }
  *out = g_dev_ptr[dev];
  return PM_OK;
}

}  // namespace

extern "C" int pm_force_static(const pm_config* cfg, const float* d_pos, int64_t np, float* d_force,
                               void* stream) {
  if (!cfg || !d_pos || !d_force) return PM_EINVAL;
  const size_t need = pm_workspace_bytes(cfg);
  if (need == 0) {
    std::fprintf(stderr, "pm_force_static: invalid configuration\n");
    return PM_EINVAL;
  }
  if (need > kScratchBytes) {
    std::fprintf(stderr,
                 "pm_force_static: this configuration needs %zu bytes of scratch, more than the %zu of the "
                 "static array; use pm_create with a workspace instead\n",
                 need, kScratchBytes);
    return PM_ENOMEM;
  }
  void* ws = nullptr;
  int s = scratch_address(&ws);
  if (s != PM_OK) return s;
  // a context over the static array: pm_create uploads the static tables
  // into it (and waits for the upload), pm_force enqueues the force; the
  // host-side context is not needed once the work is enqueued
  pm_ctx* ctx = nullptr;
  s = pm_create(cfg, ws, kScratchBytes, stream, &ctx);
  if (s != PM_OK) return s;
  s = pm_force(ctx, d_pos, np, d_force);
  if (s != PM_OK) std::fprintf(stderr, "pm_force_static: %s\n", pm_last_error(ctx));
  pm_destroy(ctx);
  return s;
}
