// Perturbation sampling (Sec. 3: W ~ N(0, Sigma); antithetic pairs as in
// Sec. 5) and the Dirac-mixture set of Method E (Sec. 5).
//
// A Philox4x32-10 block (Salmon et al., SC'11) gives four 32-bit words for a
// fixed (column, row block).  FP32 turns the block into four normals (two
// Box-Muller pairs; the single-instance sampler gives each pair its own
// thread, the batched one draws the whole block per thread), FP64 into two.
// Threads of a wave take consecutive columns, so every store is a coalesced
// 256/512-byte row segment of the sample-fastest W.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "philox.hpp"

namespace gnm {
namespace {

// Block (bx, by): draws bx * 256 + thread of the rows kRows by .. kRows by + kRows - 1.
// With `hi` / `lo` (float32 only) the draws are also written as the hi + lo
// bfloat16 planes (n x kpad, zero beyond K) that the BF16x3 contraction reads.
template <typename T>
__device__ __forceinline__ void sample_block(int n, int Kdraw, T sigma, uint32_t k0, uint32_t k1,
                                             uint32_t s0, uint32_t s1, int antithetic,
                                             T* __restrict__ W, int64_t ldw, int bx, int by,
                                             __bf16* __restrict__ hi = nullptr,
                                             __bf16* __restrict__ lo = nullptr, int kpad = 0) {
  const int s = bx * 256 + threadIdx.x;
  const int b = by;
  if (s >= Kdraw) return;
  const Philox4x32 x = philox4x32_10(Philox4x32{static_cast<uint32_t>(s), static_cast<uint32_t>(b), s0, s1}, k0, k1);
  constexpr int kRows = sizeof(T) == 4 ? 4 : 2;
  T z[kRows];
  if constexpr (sizeof(T) == 4) {
    box_muller_f32(x.c0, x.c1, z[0], z[1]);
    box_muller_f32(x.c2, x.c3, z[2], z[3]);
  } else {
    box_muller_f64(x, z[0], z[1]);
  }
  const int K = antithetic ? 2 * Kdraw : Kdraw;
#pragma unroll
  for (int t = 0; t < kRows; ++t) {
    const int row = kRows * b + t;
    if (row < n) {
      const T v = sigma * z[t];
      W[row * ldw + s] = v;
      if (antithetic) W[row * ldw + s + Kdraw] = -v;
      if constexpr (sizeof(T) == 4) {
        if (hi != nullptr) {
          const __bf16 h = static_cast<__bf16>(v);
          const __bf16 l = static_cast<__bf16>(v - static_cast<float>(h));
          const int64_t o = static_cast<int64_t>(row) * kpad;
          hi[o + s] = h;
          lo[o + s] = l;
          if (antithetic) {  // -v splits into -h and -l exactly
            hi[o + s + Kdraw] = -h;
            lo[o + s + Kdraw] = -l;
          }
          for (int pz = s; pz < kpad - K; pz += Kdraw) {  // zero padding up to kpad
            hi[o + K + pz] = __bf16(0.0f);
            lo[o + K + pz] = __bf16(0.0f);
          }
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) sample_kernel(int n, int Kdraw, T sigma, uint32_t k0,
                                                     uint32_t k1, uint32_t s0, uint32_t s1,
                                                     int antithetic, T* __restrict__ W,
                                                     int64_t ldw) {
  sample_block<T>(n, Kdraw, sigma, k0, k1, s0, s1, antithetic, W, ldw, blockIdx.x, blockIdx.y);
}

// FP32 with half the work per thread: block row y takes half y % 2 of the
// Philox block y / 2 (rows 4 (y / 2) + 2 (y % 2) and the next), the same
// numbers as sample_kernel<float>.  Twice the threads, one Box-Muller pair
// each: the sampler is latency-bound at these sizes.
__global__ void __launch_bounds__(256) sample_half_kernel(int n, int Kdraw, float sigma,
                                                          uint32_t k0, uint32_t k1, uint32_t s0,
                                                          uint32_t s1, int antithetic,
                                                          float* __restrict__ W, int64_t ldw) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y >> 1, half = blockIdx.y & 1;
  const int row0 = 4 * b + 2 * half;
  if (s >= Kdraw || row0 >= n) return;
  const Philox4x32 x = philox4x32_10(
      Philox4x32{static_cast<uint32_t>(s), static_cast<uint32_t>(b), s0, s1}, k0, k1);
  float z[2];
  if (half == 0)
    box_muller_f32(x.c0, x.c1, z[0], z[1]);
  else
    box_muller_f32(x.c2, x.c3, z[0], z[1]);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int row = row0 + t;
    if (row < n) {
      const float v = sigma * z[t];
      W[row * ldw + s] = v;
      if (antithetic) W[row * ldw + s + Kdraw] = -v;
    }
  }
}

// Batched: instance b draws with key b.seed and the stream id of the
// iteration (the same numbers as a single-instance call with that seed);
// tile = by * ceil(Kdraw / 256) + bx.
__global__ void __launch_bounds__(256) batch_sample_kernel(const BatchInst* __restrict__ inst,
                                                           BatchLaunch L, float sigma, uint32_t s0,
                                                           uint32_t s1) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    const int Kdraw = b.K / 2;
    const int xb = (Kdraw + 255) / 256;
    sample_block<float>(b.n, Kdraw, sigma, static_cast<uint32_t>(b.seed),
                        static_cast<uint32_t>(b.seed >> 32), s0, s1, 1, b.W, b.ldw, it.tile % xb,
                        it.tile / xb, b.Wh, b.Wl, b.kpad);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) sigma_points_kernel(int n, T scale, T* __restrict__ W,
                                                           int64_t ldw) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  const int row = blockIdx.y;
  if (s >= 2 * n) return;
  T v = 0;
  if (s == row) v = scale;
  if (s == row + n) v = -scale;
  W[row * ldw + s] = v;
}

}  // namespace

int batch_sample_tiles(int n, int K) { return ((K / 2 + 255) / 256) * ((n + 3) / 4); }

hipError_t launch_batch_sample(const BatchInst* inst, const BatchLaunch& L, double sigma,
                               uint64_t stream_id, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_sample_kernel, dim3(L.blocks), dim3(256), 0, st, inst, L,
                     static_cast<float>(sigma), static_cast<uint32_t>(stream_id),
                     static_cast<uint32_t>(stream_id >> 32));
  return hipGetLastError();
}

hipError_t launch_sample(int dtype, int n, int K, double sigma, uint64_t seed,
                         uint64_t stream_id, int antithetic, void* W, int64_t ldw,
                         hipStream_t st) {
  const int Kdraw = antithetic ? K / 2 : K;
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const uint32_t s0 = static_cast<uint32_t>(stream_id), s1 = static_cast<uint32_t>(stream_id >> 32);
  // two rows per block row: FP32 one Box-Muller pair of a Philox block per
  // thread, FP64 the block's two normals
  dim3 grid((Kdraw + 255) / 256, (n + 1) / 2);
  if (dtype == GNMPPI_F32)
    hipLaunchKernelGGL(sample_half_kernel, grid, dim3(256), 0, st, n, Kdraw,
                       static_cast<float>(sigma), k0, k1, s0, s1, antithetic,
                       static_cast<float*>(W), ldw);
  else
    hipLaunchKernelGGL(sample_kernel<double>, grid, dim3(256), 0, st, n, Kdraw, sigma, k0, k1,
                       s0, s1, antithetic, static_cast<double*>(W), ldw);
  return hipGetLastError();
}

hipError_t launch_sigma_points(int dtype, int n, double sigma, void* W, int64_t ldw,
                               hipStream_t st) {
  dim3 grid((2 * n + 255) / 256, n);
  const double scale = __builtin_sqrt(static_cast<double>(n)) * sigma;
  if (dtype == GNMPPI_F32)
    hipLaunchKernelGGL(sigma_points_kernel<float>, grid, dim3(256), 0, st, n,
                       static_cast<float>(scale), static_cast<float*>(W), ldw);
  else
    hipLaunchKernelGGL(sigma_points_kernel<double>, grid, dim3(256), 0, st, n, scale,
                       static_cast<double*>(W), ldw);
  return hipGetLastError();
}

}  // namespace gnm
