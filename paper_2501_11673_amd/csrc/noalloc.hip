// Device scratch of the no-allocation entry point (kpp_block_factor_noalloc).
//
// One file-scope array per device holds everything that entry point needs
// beyond its inputs and outputs: the staged block rows, lengths and slot ids,
// the breakdown flag and the split-Gram workspace.  Host code never uses the
// array's name as an address (on the host it names a stand-in, not device
// memory): noalloc_scratch() resolves the device address once per device,
// with that device current, and every later use goes through that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace kpp {
namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidValue;   // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidValue;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace kpp
