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

// ---- BF16 MFMA contraction of the residual differences -----------------------
//
// S = (R - r0 1^T) W^T with v_mfma_f32_16x16x32_bf16 and FP32 accumulation.
// TERMS = 1: A and B rounded to bf16 (the precision split: ~2^-9 relative per
// product).  TERMS = 3: each operand is split into hi + lo bf16 parts and
// S ~ Ah Bh + Ah Bl + Al Bh, which drops only the lo*lo term and the second
// rounding, so the products carry ~16 bits and the sums stay at FP32-level
// error while the MFMA rate is 16x that of v_mfma_f32_16x16x4f32.
// Layout (measured): lane l supplies A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] for e < 8; accumulator j is D[4 (l / 16) + j][l % 16].
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x4 = float __attribute__((ext_vector_type(4)));
constexpr int kBf16Step = 32;

// W (n x K, ldw) -> hi and lo bf16 planes (n x kpad), zero beyond K.
__global__ void __launch_bounds__(256) split_bf16_kernel(int K, int kpad, const float* __restrict__ W,
                                                         int64_t ldw, __bf16* __restrict__ hi,
                                                         __bf16* __restrict__ lo) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int row = blockIdx.y;
  if (k >= kpad) return;
  const float v = k < K ? W[row * ldw + k] : 0.0f;
  const __bf16 h = static_cast<__bf16>(v);
  hi[static_cast<int64_t>(row) * kpad + k] = h;
  lo[static_cast<int64_t>(row) * kpad + k] = static_cast<__bf16>(v - static_cast<float>(h));
}

template <int TERMS, int NT, bool VEC>
__global__ void __launch_bounds__(256) contract_bf16_kernel(
    int m, int n, int K, const float* __restrict__ R, int64_t ldr, const float* __restrict__ r0,
    const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl, int kpad, int split_len,
    float* __restrict__ part, int npad) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row_base = (blockIdx.x * 4 + wave) * 16;
  const int kbeg = blockIdx.y * split_len;
  const int kend = min(K, kbeg + split_len);
  const int row = row_base + r16;
  const float* arow = R + (row < m ? row : 0) * ldr;
  const float asub = row < m ? r0[row] : 0.0f;
  int64_t boff[NT];
  bool bzero[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) {
    const int col = 16 * tn + r16;
    boff[tn] = static_cast<int64_t>(col < n ? col : 0) * kpad;
    bzero[tn] = col >= n;
  }
  f32x4 acc[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) acc[tn] = f32x4{0, 0, 0, 0};
  if (row_base < m) {
    for (int k0 = kbeg; k0 < kend; k0 += kBf16Step) {
      const int kl = k0 + 8 * kq;
      float a[8];
      if (VEC && k0 + kBf16Step <= kend) {
        const f32x4 x0 = *reinterpret_cast<const f32x4*>(arow + kl);
        const f32x4 x1 = *reinterpret_cast<const f32x4*>(arow + kl + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a[e] = x0[e];
          a[4 + e] = x1[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = (kl + e < kend) ? arow[kl + e] : 0.0f;
      }
      bf16x8 ah, al;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float v = (kl + e < kend) ? a[e] - asub : 0.0f;
        ah[e] = static_cast<__bf16>(v);
        if constexpr (TERMS == 3) al[e] = static_cast<__bf16>(v - static_cast<float>(ah[e]));
      }
#pragma unroll
      for (int tn = 0; tn < NT; ++tn) {
        bf16x8 bh = *reinterpret_cast<const bf16x8*>(Bh + boff[tn] + kl);
        if (bzero[tn]) bh = bf16x8{};
        acc[tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[tn], 0, 0, 0);
        if constexpr (TERMS == 3) {
          bf16x8 bl = *reinterpret_cast<const bf16x8*>(Bl + boff[tn] + kl);
          if (bzero[tn]) bl = bf16x8{};
          acc[tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[tn], 0, 0, 0);
          acc[tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[tn], 0, 0, 0);
        }
      }
    }
  }
  float* out = part + static_cast<int64_t>(blockIdx.y) * m * npad;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int orow = row_base + 4 * kq + j;
    if (orow < m)
#pragma unroll
      for (int tn = 0; tn < NT; ++tn) out[orow * npad + 16 * tn + r16] = acc[tn][j];
  }
}

template <int TERMS, bool VEC>
hipError_t bf16_dispatch(int nt, dim3 grid, hipStream_t st, int m, int n, int K, const float* R,
                         int64_t ldr, const float* r0, const __bf16* Bh, const __bf16* Bl, int kpad,
                         int split_len, float* part, int npad) {
#define GNM_BF_CASE(NT)                                                                        \
  case NT:                                                                                     \
    hipLaunchKernelGGL((contract_bf16_kernel<TERMS, NT, VEC>), grid, dim3(256), 0, st, m, n, K, \
                       R, ldr, r0, Bh, Bl, kpad, split_len, part, npad);                       \
    break;
  switch (nt) {
    GNM_BF_CASE(1) GNM_BF_CASE(2) GNM_BF_CASE(3) GNM_BF_CASE(4) GNM_BF_CASE(5) GNM_BF_CASE(6)
    GNM_BF_CASE(7) GNM_BF_CASE(8) GNM_BF_CASE(9) GNM_BF_CASE(10) GNM_BF_CASE(11) GNM_BF_CASE(12)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_BF_CASE
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract(const ContractArgs<float>& a, int nsplit, hipStream_t st) {
  return contract_typed(a, nsplit, st);
}
hipError_t launch_contract(const ContractArgs<double>& a, int nsplit, hipStream_t st) {
  return contract_typed(a, nsplit, st);
}

hipError_t launch_split_bf16(int n, int K, int kpad, const float* W, int64_t ldw, __bf16* hi,
                             __bf16* lo, hipStream_t st) {
  hipLaunchKernelGGL(split_bf16_kernel, dim3((kpad + 255) / 256, n), dim3(256), 0, st, K, kpad, W,
                     ldw, hi, lo);
  return hipGetLastError();
}

hipError_t launch_contract_bf16(int terms, int m, int n, int K, const float* R, int64_t ldr,
                                const float* r0, const __bf16* Bh, const __bf16* Bl, int kpad,
                                int nsplit, int split_len, float* part, int npad, hipStream_t st) {
  dim3 grid((m + 63) / 64, nsplit);
  const int nt = (n + 15) / 16;
  const bool vec = (ldr % 4 == 0) && (reinterpret_cast<uintptr_t>(R) % 16 == 0);
  if (terms == 3)
    return vec ? bf16_dispatch<3, true>(nt, grid, st, m, n, K, R, ldr, r0, Bh, Bl, kpad, split_len,
                                        part, npad)
               : bf16_dispatch<3, false>(nt, grid, st, m, n, K, R, ldr, r0, Bh, Bl, kpad, split_len,
                                         part, npad);
  return vec ? bf16_dispatch<1, true>(nt, grid, st, m, n, K, R, ldr, r0, Bh, Bl, kpad, split_len,
                                      part, npad)
             : bf16_dispatch<1, false>(nt, grid, st, m, n, K, R, ldr, r0, Bh, Bl, kpad, split_len,
                                       part, npad);
}

}  // namespace gnm
