// Device memory of the allocation-free entry point (fcc_tdoa_noalloc): one
// file-scope array per GPU, created with the code object and held until the
// process ends.  Its host-side name is not a device address; the address each
// device holds is fetched once per device, with that device current, and that
// pointer is the only way host code reaches the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fcc.h"
#include "kernels.hpp"

static __device__ __align__(256) unsigned char scratch[FCC_NOALLOC_SCRATCH_BYTES];

namespace fcc {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace fcc
