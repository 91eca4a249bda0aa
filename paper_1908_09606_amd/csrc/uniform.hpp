// Values that are the same in every lane of a wave, read through the first
// lane so that they stay in scalar registers instead of one vector register
// per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cosma {

__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const int lo = __builtin_amdgcn_readfirstlane((int)x);
  const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform_i64(reinterpret_cast<int64_t>(p)));
}
__device__ __forceinline__ double uniform_f64(double x) {
  return __builtin_bit_cast(double, uniform_i64(__builtin_bit_cast(int64_t, x)));
}

}  // namespace cosma
