// Accumulator element types: binary32 (default) or, to measure accumulation
// stagnation, bfloat16 / binary16 (round to nearest even on every update).
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

template <int AT>
__device__ __forceinline__ float acc_load(const void* A, int64_t i) {
  if constexpr (AT == 0) return reinterpret_cast<const float*>(A)[i];
  else if constexpr (AT == 1) return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(A)[i]);
  else return __half2float(reinterpret_cast<const __half*>(A)[i]);
}

template <int AT>
__device__ __forceinline__ void acc_store(void* A, int64_t i, float v) {
  if constexpr (AT == 0) reinterpret_cast<float*>(A)[i] = v;
  else if constexpr (AT == 1) reinterpret_cast<__hip_bfloat16*>(A)[i] = __float2bfloat16(v);
  else reinterpret_cast<__half*>(A)[i] = __float2half(v);
}

// Hardware atomic add; 16-bit elements use the packed 2x16-bit atomic with a
// zero in the neighbouring half.
template <int AT>
__device__ __forceinline__ void acc_atomic_add(void* A, int64_t i, float v) {
  if constexpr (AT == 0) unsafeAtomicAdd(reinterpret_cast<float*>(A) + i, v);
  else if constexpr (AT == 1) unsafeAtomicAdd(reinterpret_cast<__hip_bfloat16*>(A) + i, __float2bfloat16(v));
  else unsafeAtomicAdd(reinterpret_cast<__half*>(A) + i, __float2half(v));
}

}  // namespace lf
