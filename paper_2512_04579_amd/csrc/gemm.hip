// Contractions of the form  out = A B^T  with the contraction index
// contiguous in both operands, on MFMA.  The Jacobian reconstruction of
// Eq. (10) uses it twice: S = (R - r0 1^T) W^T and G = W W^T over the sample
// index, then J = S G^{-1} over the decision index (G^{-1} is symmetric).
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
__global__ void __launch_bounds__(256) contract_kernel(ContractArgs<T> a) {
  using MT = Mfma<T>;
  using Acc = typename MT::Acc;
  constexpr int V = MT::kLaneK, STEP = MT::kStep;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row_base = (blockIdx.x * 4 + wave) * 16 * TM;
  const int kbeg = blockIdx.y * a.split_len;
  const int kend = min(a.K, kbeg + a.split_len);

  const T* arow[TM];
  T asub[TM];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm) {
    const int row = row_base + 16 * tm + r16;
    if (row < a.m) {
      arow[tm] = a.A + row * a.lda;
      asub[tm] = a.asub ? a.asub[row] : T(0);
    } else if (row < a.rows) {
      arow[tm] = a.A2 + (row - a.m) * a.lda2;
      asub[tm] = 0;
    } else {  // past the last row: read a valid row, never stored
      arow[tm] = a.B;
      asub[tm] = 0;
    }
  }
  const T* bcol[NT];
  bool bzero[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) {
    const int col = 16 * tn + r16;
    bcol[tn] = a.B + (col < a.ncol ? col : 0) * a.ldb;
    bzero[tn] = col >= a.ncol;
  }

  Acc acc[TM][NT];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < NT; ++tn) acc[tm][tn] = Acc{0, 0, 0, 0};

  if (row_base < a.rows) {
    for (int k0 = kbeg; k0 < kend; k0 += STEP) {
      const bool full = k0 + STEP <= kend;
      const int kl = k0 + kq * V;
      T av[TM][V], bv[NT][V];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        load_lane_k<T, VEC>(arow[tm], kl, kend, full, av[tm]);
#pragma unroll
        for (int t = 0; t < V; ++t) av[tm][t] = (kl + t < kend) ? av[tm][t] - asub[tm] : T(0);
      }
#pragma unroll
      for (int tn = 0; tn < NT; ++tn) {
        load_lane_k<T, VEC>(bcol[tn], kl, kend, full, bv[tn]);
        if (bzero[tn])
#pragma unroll
          for (int t = 0; t < V; ++t) bv[tn][t] = 0;
      }
#pragma unroll
      for (int t = 0; t < V; ++t)
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < NT; ++tn) acc[tm][tn] = MT::mma(av[tm][t], bv[tn][t], acc[tm][tn]);
    }
  }

  T* out = a.out + static_cast<int64_t>(blockIdx.y) * a.split_stride;
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row_base + 16 * tm + MT::out_row(kq, j);
      if (row < a.rows)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn) {
          const int col = 16 * tn + r16;
          if (col < a.ocols) out[row * a.ldo + col] = acc[tm][tn][j];
        }
    }
}

template <typename T, int TM, bool VEC>
hipError_t contract_dispatch_nt(int nt, dim3 grid, hipStream_t st, const ContractArgs<T>& a) {
#define GNM_NT_CASE(NT)                                                                       \
  case NT:                                                                                    \
    hipLaunchKernelGGL((contract_kernel<T, TM, NT, VEC>), grid, dim3(256), 0, st, a);         \
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

template <typename T>
bool vec_ok(const T* p, int64_t ld) {
  constexpr int per = 16 / sizeof(T);
  return p == nullptr || ((ld % per) == 0 && (reinterpret_cast<uintptr_t>(p) % 16) == 0);
}

template <typename T>
hipError_t contract_typed(const ContractArgs<T>& a, int nsplit, hipStream_t st) {
  constexpr int TM = 1;
  const int row_blocks = (a.rows + 64 * TM - 1) / (64 * TM);
  dim3 grid(row_blocks, nsplit);
  const int nt = (a.ncol + 15) / 16;
  const bool vec = vec_ok(a.A, a.lda) && vec_ok(a.A2, a.lda2) && vec_ok(a.B, a.ldb);
  if (vec) return contract_dispatch_nt<T, TM, true>(nt, grid, st, a);
  return contract_dispatch_nt<T, TM, false>(nt, grid, st, a);
}

}  // namespace

hipError_t launch_contract(const ContractArgs<float>& a, int nsplit, hipStream_t st) {
  return contract_typed(a, nsplit, st);
}
hipError_t launch_contract(const ContractArgs<double>& a, int nsplit, hipStream_t st) {
  return contract_typed(a, nsplit, st);
}

}  // namespace gnm
