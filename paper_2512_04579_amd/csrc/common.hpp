// Device-side helpers shared by the GN-MPPI kernels (gfx950, wave64).
#pragma once
#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gnmppi.h"

namespace gnm {

constexpr int kWave = 64;

// ---- lane shifts inside 16-lane DPP rows --------------------------------
// row_shr:1 -> lane l reads lane l-1 of its row (row lane 0 reads 0);
// row_shl:1 -> lane l reads lane l+1 of its row (row lane 15 reads 0).
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShl1 = 0x101;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(b)), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(b >> 32)), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                        static_cast<uint32_t>(lo));
}

// ---- reductions ----------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T o = __shfl_xor(v, off, kWave);
    v = o < v ? o : v;
  }
  return v;
}

// Block-wide reductions; `scratch` holds one slot per wave (<= 16 waves).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T t = 0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  return t;
}

template <typename T>
__device__ __forceinline__ T block_min(T v, T* scratch) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_min(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T t = scratch[0];
  for (int w = 1; w < nw; ++w) t = scratch[w] < t ? scratch[w] : t;
  return t;
}

template <typename T>
__device__ __forceinline__ bool finite(T v) {
  return __builtin_isfinite(v);
}

template <typename T>
__device__ __forceinline__ T infinity() {
  return __builtin_huge_val();
}
template <>
__device__ __forceinline__ float infinity<float>() {
  return __builtin_huge_valf();
}

__device__ __forceinline__ float dsqrt(float v) { return __builtin_sqrtf(v); }
__device__ __forceinline__ double dsqrt(double v) { return __builtin_sqrt(v); }

// f(std::integral_constant<int, S>{}) for S = B .. E - 1, so that the body
// sees its index as a constant expression.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

}  // namespace gnm
