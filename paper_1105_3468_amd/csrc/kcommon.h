// Device-side helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gmg {

// "Not yet computed" marker of the synchronisation-free sweeps: a quiet NaN
// with a payload no arithmetic produces (arithmetic NaNs are the canonical
// 0x7ff8000000000000 / 0x7fc00000 or carry an input NaN's payload, and inputs
// are checked to be finite).
constexpr uint64_t SENT64 = 0x7FF8DEADBEEFF00DULL;
constexpr uint32_t SENT32 = 0x7FC0FEEDu;

template <class T>
__device__ __forceinline__ T sentinel_of(uint64_t);
template <>
__device__ __forceinline__ double sentinel_of<double>(uint64_t) { return __builtin_bit_cast(double, SENT64); }
template <>
__device__ __forceinline__ float sentinel_of<float>(uint64_t) { return __builtin_bit_cast(float, SENT32); }

__device__ __forceinline__ bool is_sentinel(double v) { return __builtin_bit_cast(uint64_t, v) == SENT64; }
__device__ __forceinline__ bool is_sentinel(float v) { return __builtin_bit_cast(uint32_t, v) == SENT32; }

// Relaxed agent-scope accesses: coherent across the XCDs' L2 caches without a
// cache-wide write-back or invalidate (no release/acquire fences).
template <class T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace gmg
