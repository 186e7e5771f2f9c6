// noalloc.hip -- the static device scratch of the entry point that allocates
// nothing (fbg_enumerate_noalloc): the enumeration's temporaries (per-tile
// model counts, their exclusive scan, block sums) live in one file-scope
// device array of fixed size instead of a stream-ordered allocation.  Every
// device the library runs on holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fbg_kernels.h"

namespace fbg {

namespace {

static __device__ __align__(256) uint64_t scratch[kNoallocScratchBytes / sizeof(uint64_t)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // the array's device address on each device, once looked up

}  // namespace

// The device address of `scratch` on the current device (looked up once per
// device with that device current; host code must never pass the array's
// own name to a kernel, which is a host-side stand-in).
hipError_t noalloc_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace fbg
