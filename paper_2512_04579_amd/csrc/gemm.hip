// Contractions over the sample index for the Jacobian reconstruction of
// Eq. (10):  S = (R - r0 1^T) W^T  (m x n)  and  G = W W^T  (n x n).
//
// Both operands are sample-fastest, so the contraction index is the
// contiguous one for A and for B ("A B^T" form): each lane streams 16-byte
// vectors straight from HBM into MFMA operands.  The two products share B,
// so they run as one launch over the stacked row set [R rows ; W rows]; the
// nominal-residual subtraction is fused into the A-operand load.
//
// Work split: a wave owns 16*TM output rows and all n output columns (n <=
// 192 -> up to 12 16-column MFMA tiles); the four waves of a block own
// adjacent row tiles and read the same W columns, which therefore hit in L1.
// The sample range is cut into `nsplit` slices (grid.y) so that ~1.5k waves
// cover the machine; each slice writes its own partial sum and the consumer
// kernels add the slices in a fixed order (bitwise reproducible results).
//
// MFMA operand layout (16x16x4, both f32 and f64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator element j of lane l
// is D[4 (l / 16) + j][l % 16] for f32 but D[4 j + l / 16][l % 16] for f64
// (measured with a one-wave probe).  A lane that loads k-values kl..kl+V-1 feeds
// them to V consecutive MFMAs; the k-permutation this induces is the same
// for A and B, so the sum is unchanged.
#include "common.hpp"
#include "launch.hpp"

namespace gnm {
namespace {

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  using Acc = float __attribute__((ext_vector_type(4)));
  using Vec = float __attribute__((ext_vector_type(4)));
  static constexpr int kLaneK = 8;  // k-values per lane per step (two 16-byte loads)
  static constexpr int kStep = 32;  // 4 lane groups x kLaneK
  static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of accumulator element j held by lane group kq = lane / 16
  static __device__ __forceinline__ int out_row(int kq, int j) { return 4 * kq + j; }
};

template <>
struct Mfma<double> {
  using Acc = double __attribute__((ext_vector_type(4)));
  using Vec = double __attribute__((ext_vector_type(2)));
  static constexpr int kLaneK = 4;
  static constexpr int kStep = 16;
  static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int kq, int j) { return 4 * j + kq; }
};

template <typename T, bool VEC>
__device__ __forceinline__ void load_lane_k(const T* __restrict__ p, int kl, int kend, bool full,
                                            T (&v)[Mfma<T>::kLaneK]) {
  constexpr int V = Mfma<T>::kLaneK;
  if (VEC && full) {
    using Vec = typename Mfma<T>::Vec;
    constexpr int per = sizeof(Vec) / sizeof(T);
#pragma unroll
    for (int h = 0; h < V / per; ++h) {
      const Vec x = *reinterpret_cast<const Vec*>(p + kl + h * per);
#pragma unroll
      for (int e = 0; e < per; ++e) v[h * per + e] = x[e];
    }
  } else {
#pragma unroll
    for (int t = 0; t < V; ++t) v[t] = (kl + t < kend) ? p[kl + t] : T(0);
  }
}

template <typename T, int TM, int NT, bool VEC>
__global__ void __launch_bounds__(256) jac_contract_kernel(
    int m, int n, int rows, int K, const T* __restrict__ R, int64_t ldr, const T* __restrict__ r0,
    const T* __restrict__ W, int64_t ldw, int split_len, T* __restrict__ part, int npad) {
  using MT = Mfma<T>;
  using Acc = typename MT::Acc;
  constexpr int V = MT::kLaneK, STEP = MT::kStep;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row_base = (blockIdx.x * 4 + wave) * 16 * TM;
  const int kbeg = blockIdx.y * split_len;
  const int kend = min(K, kbeg + split_len);

  const T* arow[TM];
  T asub[TM];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm) {
    const int row = row_base + 16 * tm + r16;
    if (row < m) {
      arow[tm] = R + row * ldr;
      asub[tm] = r0[row];
    } else if (row < rows) {
      arow[tm] = W + (row - m) * ldw;
      asub[tm] = 0;
    } else {  // past the last row: read a valid row, never stored
      arow[tm] = W;
      asub[tm] = 0;
    }
  }
  const T* bcol[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) {
    const int col = 16 * tn + r16;
    bcol[tn] = W + (col < n ? col : 0) * ldw;
  }
  bool bzero[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) bzero[tn] = (16 * tn + r16) >= n;

  Acc acc[TM][NT];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < NT; ++tn) acc[tm][tn] = Acc{0, 0, 0, 0};

  if (row_base < rows) {
    for (int k0 = kbeg; k0 < kend; k0 += STEP) {
      const bool full = k0 + STEP <= kend;
      const int kl = k0 + kq * V;
      T a[TM][V], b[NT][V];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        load_lane_k<T, VEC>(arow[tm], kl, kend, full, a[tm]);
#pragma unroll
        for (int t = 0; t < V; ++t) a[tm][t] = (kl + t < kend) ? a[tm][t] - asub[tm] : T(0);
      }
#pragma unroll
      for (int tn = 0; tn < NT; ++tn) {
        load_lane_k<T, VEC>(bcol[tn], kl, kend, full, b[tn]);
        if (bzero[tn])
#pragma unroll
          for (int t = 0; t < V; ++t) b[tn][t] = 0;
      }
#pragma unroll
      for (int t = 0; t < V; ++t)
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < NT; ++tn) acc[tm][tn] = MT::mma(a[tm][t], b[tn][t], acc[tm][tn]);
    }
  }

  T* out = part + static_cast<int64_t>(blockIdx.y) * rows * npad;
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row_base + 16 * tm + MT::out_row(kq, j);
      if (row < rows)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn) out[row * npad + 16 * tn + r16] = acc[tm][tn][j];
    }
}

template <typename T, int TM, bool VEC>
hipError_t contract_dispatch_nt(int nt, dim3 grid, hipStream_t st, int m, int n, int rows, int K,
                                const T* R, int64_t ldr, const T* r0, const T* W, int64_t ldw,
                                int split_len, T* part, int npad) {
#define GNM_NT_CASE(NT)                                                                           \
  case NT:                                                                                        \
    hipLaunchKernelGGL((jac_contract_kernel<T, TM, NT, VEC>), grid, dim3(256), 0, st, m, n, rows, \
                       K, R, ldr, r0, W, ldw, split_len, part, npad);                             \
    break;
  switch (nt) {
    GNM_NT_CASE(1) GNM_NT_CASE(2) GNM_NT_CASE(3) GNM_NT_CASE(4) GNM_NT_CASE(5) GNM_NT_CASE(6)
    GNM_NT_CASE(7) GNM_NT_CASE(8) GNM_NT_CASE(9) GNM_NT_CASE(10) GNM_NT_CASE(11) GNM_NT_CASE(12)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_NT_CASE
  return hipGetLastError();
}

}  // namespace

// Shared by the Jacobian launcher in dense.hip.
hipError_t launch_jac_contract(int dtype, int m, int n, int rows, int K, const void* R,
                               int64_t ldr, const void* r0, const void* W, int64_t ldw,
                               int nsplit, int split_len, void* part, int npad, hipStream_t st) {
  constexpr int TM = 1;
  const int row_blocks = (rows + 64 * TM - 1) / (64 * TM);
  dim3 grid(row_blocks, nsplit);
  const int nt = npad / 16;
  if (dtype == GNMPPI_F32) {
    const float* Rf = static_cast<const float*>(R);
    const float* Wf = static_cast<const float*>(W);
    const bool vec = (ldr % 4 == 0) && (ldw % 4 == 0) &&
                     (reinterpret_cast<uintptr_t>(Rf) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(Wf) % 16 == 0);
    if (vec)
      return contract_dispatch_nt<float, TM, true>(nt, grid, st, m, n, rows, K, Rf, ldr,
                                                   static_cast<const float*>(r0), Wf, ldw,
                                                   split_len, static_cast<float*>(part), npad);
    return contract_dispatch_nt<float, TM, false>(nt, grid, st, m, n, rows, K, Rf, ldr,
                                                  static_cast<const float*>(r0), Wf, ldw,
                                                  split_len, static_cast<float*>(part), npad);
  }
  const double* Rd = static_cast<const double*>(R);
  const double* Wd = static_cast<const double*>(W);
  const bool vec = (ldr % 2 == 0) && (ldw % 2 == 0) &&
                   (reinterpret_cast<uintptr_t>(Rd) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(Wd) % 16 == 0);
  if (vec)
    return contract_dispatch_nt<double, TM, true>(nt, grid, st, m, n, rows, K, Rd, ldr,
                                                  static_cast<const double*>(r0), Wd, ldw,
                                                  split_len, static_cast<double*>(part), npad);
  return contract_dispatch_nt<double, TM, false>(nt, grid, st, m, n, rows, K, Rd, ldr,
                                                 static_cast<const double*>(r0), Wd, ldw,
                                                 split_len, static_cast<double*>(part), npad);
}

}  // namespace gnm
