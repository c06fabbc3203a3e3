// Library-owned device scratch for the entry point that allocates nothing
// (mra_loglik_grad_noalloc): a file-scope device array that every GPU the
// library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel or a copy (in host code it is a host-side
// stand-in, not a device address): it looks up the array's device address
// once per device with hipGetSymbolAddress and hands that pointer out.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mra.h"

namespace mra {
namespace {

static_assert(MRA_NOALLOC_MAX_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) double scratch[MRA_NOALLOC_MAX_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Device address of the scratch array on the current device, looked up on
// the first call for that device (with the device current) and kept.
hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidValue;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace mra
