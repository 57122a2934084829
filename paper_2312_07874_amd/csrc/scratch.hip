// Library-owned residual workspace for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation): a file-scope device array of fixed size, one copy per
// GPU, held until the process ends.
//
// In host code the array's name is only a host-side stand-in; its device
// address is looked up with hipGetSymbolAddress once per device (with that
// device current) and kept, and only that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scratch.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[esd::SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_addr[MAX_DEVICES] = {};

}  // namespace

namespace esd {

int scratch_address(void** out, int* device) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  if (device) *device = dev;
  return 0;
}

}  // namespace esd
