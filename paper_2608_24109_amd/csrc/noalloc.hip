// Device scratch of the entry point that allocates nothing (exm_shade_fwd_noalloc): a file-scope
// device array, one copy per GPU the library runs on, held until the process ends. Host code never
// passes the array's name to a kernel (on the host it names a stand-in, not device memory); it
// looks up each device's address once with hipGetSymbolAddress, with that device current, and
// hands that pointer to the pass as its workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  *ptr = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace exm
