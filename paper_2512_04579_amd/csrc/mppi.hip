// MPPI weighted-mean update, Eqs. (7)-(8).
//
// Every block recomputes the (cheap, K-long) weight vector into LDS -- a min
// reduction of the costs, one exp per sample and a sum -- so the update needs
// a single launch and no grid-wide synchronisation.  Each wave then owns
// whole rows of W and forms sum_s w_s W[i, s] with coalesced row loads and a
// shuffle reduction.  HBM traffic is one pass over W (n K elements) plus K
// costs per block from L2.
#include "common.hpp"
#include "launch.hpp"

namespace gnm {
namespace {

constexpr int kMppiThreads = 256;
constexpr int kMppiWaves = kMppiThreads / kWave;

template <typename T>
__global__ void __launch_bounds__(kMppiThreads) mppi_update_kernel(
    int n, int K, const T* __restrict__ C, const T* __restrict__ W, int64_t ldw, T temperature,
    T* __restrict__ U, T* __restrict__ weights, int32_t* status) {
  extern __shared__ unsigned char smem_raw[];
  T* w = reinterpret_cast<T*>(smem_raw);
  __shared__ T red[16];
  const int tid = threadIdx.x;

  T cmin = infinity<T>();
  for (int s = tid; s < K; s += kMppiThreads) {
    const T c = C[s];
    if (finite(c) && c < cmin) cmin = c;
  }
  cmin = block_min(cmin, red);
  if (!finite(cmin)) {  // no finite cost: leave U untouched
    if (blockIdx.x == 0 && tid == 0 && status) *status = GNMPPI_ENONFINITE;
    return;
  }
  T z = 0;
  for (int s = tid; s < K; s += kMppiThreads) {
    const T c = C[s];
    const T ws = finite(c) ? exp(-(c - cmin) / temperature) : T(0);
    w[s] = ws;
    z += ws;
  }
  z = block_sum(z, red);  // contains the barrier that publishes w[]
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  for (int row = blockIdx.x * kMppiWaves + wave; row < n; row += gridDim.x * kMppiWaves) {
    const T* wr = W + row * ldw;
    T acc = 0;
    for (int s = lane; s < K; s += kWave) acc += w[s] * wr[s];
    acc = wave_sum(acc);
    if (lane == 0) U[row] = U[row] + acc / z;
  }
  if (blockIdx.x == 0) {
    if (weights)
      for (int s = tid; s < K; s += kMppiThreads) weights[s] = w[s] / z;
    if (tid == 0 && status) *status = GNMPPI_OK;
  }
}

}  // namespace

hipError_t launch_mppi_update(int dtype, int n, int K, const void* C, const void* W, int64_t ldw,
                              double temperature, void* U, void* weights, int32_t* status,
                              hipStream_t st) {
  const int blocks = (n + kMppiWaves - 1) / kMppiWaves;
  if (dtype == GNMPPI_F32) {
    const size_t lds = static_cast<size_t>(K) * sizeof(float);
    hipLaunchKernelGGL(mppi_update_kernel<float>, dim3(blocks), dim3(kMppiThreads), lds, st, n,
                       K, static_cast<const float*>(C), static_cast<const float*>(W), ldw,
                       static_cast<float>(temperature), static_cast<float*>(U),
                       static_cast<float*>(weights), status);
  } else {
    const size_t lds = static_cast<size_t>(K) * sizeof(double);
    hipLaunchKernelGGL(mppi_update_kernel<double>, dim3(blocks), dim3(kMppiThreads), lds, st, n,
                       K, static_cast<const double*>(C), static_cast<const double*>(W), ldw,
                       temperature, static_cast<double*>(U), static_cast<double*>(weights),
                       status);
  }
  return hipGetLastError();
}

}  // namespace gnm
