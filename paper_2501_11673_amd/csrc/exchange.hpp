// Exchange between the workgroups of one persistent launch (gfx950): data
// through agent-scope relaxed atomics (they complete at the device's
// coherence point and bypass the non-coherent caches), flags that carry the
// step's epoch.  A wave publishes its stores, waits for their completion and
// then raises its flag; readers poll the flag and read the data with
// agent-scope loads.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kpp {

__device__ __forceinline__ double ld_coherent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_flag(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Raise a flag after this wave's agent-scope data stores: waiting for their
// completion orders them before the flag (a release store would in addition
// write back every dirty line of this die's L2, on every step, for data the
// kernels never publish through plain stores).
__device__ __forceinline__ void st_flag_after_stores(uint32_t* p, uint32_t v) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace kpp
