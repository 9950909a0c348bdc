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
#include <type_traits>

#include "batch.hpp"
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

// Epilogue shared by the contraction kernels.  Block = 4 waves = (4 / KW)
// row tiles of 16 rows, each worked by KW waves that take turns over the
// slice's k-steps (wave kw owns steps kw, kw + KW, ...).  With KW > 1 every
// wave parks its accumulators in LDS and the tile's 64 KW threads add the KW
// partial tiles in a fixed order (reproducible) and store whole rows
// (coalesced); with KW = 1 each lane stores its accumulators directly.
template <typename T, typename Acc, int NT, int KW, typename OutRow>
__device__ __forceinline__ void store_tiles(const Acc (&acc)[NT], T* __restrict__ lds, int row_base,
                                            int rows, T* __restrict__ out, int64_t ldo, int ocols,
                                            OutRow out_row) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  if constexpr (KW == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row_base + out_row(kq, j);
      if (row < rows)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn) {
          const int col = 16 * tn + r16;
          if (col < ocols) out[row * ldo + col] = acc[tn][j];
        }
    }
  } else {
    constexpr int LD = 16 * NT + 1;  // odd stride: lane groups land on distinct banks
    T* mine = lds + wave * 16 * LD;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int tn = 0; tn < NT; ++tn) mine[out_row(kq, j) * LD + 16 * tn + r16] = acc[tn][j];
    __syncthreads();
    const int rt = wave / KW, t = threadIdx.x - rt * KW * kWave;
    const T* tile = lds + rt * KW * 16 * LD;
    for (int e = t; e < 16 * 16 * NT; e += KW * kWave) {
      const int r = e / (16 * NT), c = e - r * (16 * NT);
      const int row = row_base + r;
      if (row < rows && c < ocols) {
        T v = tile[r * LD + c];
#pragma unroll
        for (int w = 1; w < KW; ++w) v += tile[w * 16 * LD + r * LD + c];
        out[row * ldo + c] = v;
      }
    }
  }
}

template <typename T, int NT, bool VEC, int KW>
__device__ __forceinline__ void contract_block(const ContractArgs<T>& a, int bx, int by,
                                               unsigned char* contract_smem) {
  using MT = Mfma<T>;
  using Acc = typename MT::Acc;
  constexpr int V = MT::kLaneK, STEP = MT::kStep;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row_base = (bx * (4 / KW) + wave / KW) * 16;
  const int kw = wave % KW;
  const int kbeg = by * a.split_len;
  const int kend = min(a.K, kbeg + a.split_len);

  const int row = row_base + r16;
  const T* arow;
  T asub = 0;
  int nsum = 1;  // partials added while loading (rows of A only)
  if (row < a.m) {
    arow = a.A + row * a.lda;
    asub = a.asub ? a.asub[row] : T(0);
    nsum = a.asplit;
  } else if (row < a.rows) {
    arow = a.A2 + (row - a.m) * a.lda2;
  } else {  // past the last row: read row 0 of A (present in every partial), never stored
    arow = a.m > 0 ? a.A : a.A2;
    nsum = a.m > 0 ? a.asplit : 1;
  }
  const T* bcol[NT];
  bool bzero[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) {
    const int col = 16 * tn + r16;
    bcol[tn] = a.B + (col < a.ncol ? col : 0) * a.ldb;
    bzero[tn] = col >= a.ncol;
  }

  Acc acc[NT];
#pragma unroll
  for (int tn = 0; tn < NT; ++tn) acc[tn] = Acc{0, 0, 0, 0};

  if (row_base < a.rows) {
    for (int k0 = kbeg + kw * STEP; k0 < kend; k0 += KW * STEP) {
      const bool full = k0 + STEP <= kend;
      const int kl = k0 + kq * V;
      T av[V], bv[NT][V];
      load_lane_k<T, VEC>(arow, kl, kend, full, av);
      for (int sp = 1; sp < nsum; ++sp) {
        T part[V];
        load_lane_k<T, VEC>(arow + sp * a.asplit_stride, kl, kend, full, part);
#pragma unroll
        for (int t = 0; t < V; ++t) av[t] += part[t];
      }
#pragma unroll
      for (int t = 0; t < V; ++t) av[t] = (kl + t < kend) ? av[t] - asub : T(0);
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
        for (int tn = 0; tn < NT; ++tn) acc[tn] = MT::mma(av[t], bv[tn][t], acc[tn]);
    }
  }

  if (a.status != nullptr && bx == 0 && by == 0 && threadIdx.x == 0) *a.status = GNMPPI_OK;
  T* out = a.out + static_cast<int64_t>(by) * a.split_stride;
  store_tiles<T, Acc, NT, KW>(acc, reinterpret_cast<T*>(contract_smem), row_base, a.rows, out,
                              a.ldo, a.ocols, [](int q, int j) { return MT::out_row(q, j); });
}

template <typename T, int NT, bool VEC, int KW>
__global__ void __launch_bounds__(256) contract_kernel(ContractArgs<T> a) {
  extern __shared__ unsigned char contract_smem[];
  contract_block<T, NT, VEC, KW>(a, blockIdx.x, blockIdx.y, contract_smem);
}

// Batched G = W W^T partials of an iteration (K = samples, few rows): four
// waves split the k-steps of one 16-row tile.  tile = by * row_blocks + bx.
__device__ __forceinline__ ContractArgs<float> batch_gram_w_args(const BatchInst& b) {
  return ContractArgs<float>{b.n, b.n, b.n, b.K, b.W, b.ldw, nullptr, nullptr, 0, b.W, b.ldw,
                             b.gsplit_len, b.gpart, b.npad,
                             static_cast<int64_t>(b.n) * b.npad, b.npad};
}

template <int NT>
__global__ void __launch_bounds__(256) batch_contract_kernel(const BatchInst* __restrict__ inst,
                                                             BatchLaunch L) {
  constexpr int KW = 4;
  extern __shared__ unsigned char contract_smem[];
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const ContractArgs<float> a = batch_gram_w_args(inst[it.inst]);
    const int rb = (a.rows + 64 / KW - 1) / (64 / KW);
    contract_block<float, NT, true, KW>(a, it.tile % rb, it.tile / rb, contract_smem);
    __syncthreads();  // the next item reuses the LDS
  }
}

template <typename T, int NT>
constexpr size_t split_lds_bytes() {
  return static_cast<size_t>(4) * 16 * (16 * NT + 1) * sizeof(T);
}

template <typename T, bool VEC, int KW>
hipError_t contract_dispatch_nt(int nt, dim3 grid, hipStream_t st, const ContractArgs<T>& a) {
#define GNM_NT_CASE(NT)                                                                       \
  case NT:                                                                                    \
    hipLaunchKernelGGL((contract_kernel<T, NT, VEC, KW>), grid, dim3(256),                    \
                       (KW > 1 ? split_lds_bytes<T, NT>() : size_t{0}), st, a);               \
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

template <typename T, int KW>
hipError_t contract_kw_typed(const ContractArgs<T>& a, int nsplit, hipStream_t st) {
  const int row_blocks = (a.rows + 64 / KW - 1) / (64 / KW);
  dim3 grid(row_blocks, nsplit);
  const int nt = (a.ncol + 15) / 16;
  const bool vec = vec_ok(a.A, a.lda) && vec_ok(a.A2, a.lda2) && vec_ok(a.B, a.ldb);
  if (vec) return contract_dispatch_nt<T, true, KW>(nt, grid, st, a);
  return contract_dispatch_nt<T, false, KW>(nt, grid, st, a);
}

template <typename T>
hipError_t contract_typed(const ContractArgs<T>& a, int nsplit, hipStream_t st) {
  if (contract_kw(sizeof(T), a.ncol) == 4) return contract_kw_typed<T, 4>(a, nsplit, st);
  return contract_kw_typed<T, 1>(a, nsplit, st);
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

// W (n x K, ldw) -> hi and lo bf16 planes (n x kpad), zero beyond K (the
// batched form's planes; a single launch splits W inside the contraction).
__device__ __forceinline__ void split_bf16_block(int K, int kpad, const float* __restrict__ W,
                                                 int64_t ldw, __bf16* __restrict__ hi,
                                                 __bf16* __restrict__ lo, int bx, int row) {
  const int k = bx * 256 + threadIdx.x;
  if (k >= kpad) return;
  const float v = k < K ? W[row * ldw + k] : 0.0f;
  const __bf16 h = static_cast<__bf16>(v);
  hi[static_cast<int64_t>(row) * kpad + k] = h;
  lo[static_cast<int64_t>(row) * kpad + k] = static_cast<__bf16>(v - static_cast<float>(h));
}

// Batched: tile = row * ceil(kpad / 256) + k-chunk.
__global__ void __launch_bounds__(256) batch_split_bf16_kernel(const BatchInst* __restrict__ inst,
                                                               BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    const int xb = (b.kpad + 255) / 256;
    split_bf16_block(b.K, b.kpad, b.W, b.ldw, b.Wh, b.Wl, it.tile % xb, it.tile / xb);
  }
}

// Block = 4 waves over 64 TM rows and one k-slice.  The B operand of each
// 32-wide k-step (NT 16 columns, hi and lo planes) is copied once per block
// into a double-buffered LDS stage and read by all four waves, so the L2 ->
// CU traffic for B is a quarter of what per-wave loads would move; the LDS
// stage is laid out [plane][k-group of 8][column] so that the 16 lanes of a
// fragment read 256 contiguous bytes.  The A operand (fp32 residual rows)
// streams from HBM into a ring of kBf16Depth register buffers (kept raw until
// its step), is shifted by r0 and converted to bf16 (and split into hi + lo)
// in registers; B is fetched two steps ahead into two register buffers and
// written to LDS at the end of the step before its use.  One barrier per step.
//
// Every global load is unconditional: a load whose k-group lies past the end
// of the slice reads the slice's first group instead (zeroed where it is
// converted; that group lies inside the row even when the slice holds fewer
// than 32 values), and the loop runs a whole number of ring turns, the steps
// past the slice contributing zeros.  Loads are then counted in program order, so
// each step waits only for its own data and not for the ones in flight
// behind it.
//
// VEC: 16-byte loads of 8 consecutive values of A (and of W with WF32);
// needs 16-byte aligned rows whose allocation holds whole 8-value groups
// (K % 8 == 0 for the single-instance layout; the batched rows are padded to
// 64 values).  Otherwise one clamped load per value.
//
// WF32: B comes from the FP32 W itself (Wf, leading dimension ldw; Bh, Bl
// unused) and is rounded (TERMS = 1) or split into hi + lo (TERMS = 3) on its
// way into LDS -- the same arithmetic as the split pass, without it.  Without
// WF32, B comes from the bf16 planes (Bh, Bl: n x kpad, zero past K).
using f32x8 = float __attribute__((ext_vector_type(8)));
// With WF32, rows m .. arows - 1 of A are the rows of W (Wf, no r0 shift),
// so that the same launch also forms the partials of G = W W^T.
template <int TERMS, int NT, int TM, bool VEC, bool WF32 = false>
__device__ __forceinline__ void contract_bf16_block(
    int m, int n, int K, const float* __restrict__ R, int64_t ldr, const float* __restrict__ r0,
    const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl, int kpad, int split_len,
    float* __restrict__ part, int npad, int bx, int by, const float* __restrict__ Wf = nullptr,
    int64_t ldw = 0, int arows = -1) {
  if (!WF32 || arows < m) arows = m;
  constexpr int PLANES = TERMS == 3 ? 2 : 1;
  constexpr int NCOL = 16 * NT;
  constexpr int D = kBf16Depth;
  static_assert(D % 2 == 0, "the ring turn covers both B buffers");
  // pieces per stage: 16-byte bf16 pieces of each plane, or 8-value FP32
  // pieces that yield both planes
  constexpr int CHUNKS = (WF32 ? 1 : PLANES) * NCOL * (kBf16Step / 8);
  constexpr int PER_THREAD = (CHUNKS + 255) / 256;
  using BReg = std::conditional_t<WF32, f32x8, bf16x8>;
  __shared__ bf16x8 stage[2][PLANES][kBf16Step / 8][NCOL];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row_base = bx * 64 * TM + wave * 16 * TM;
  const int kbeg = by * split_len;
  const int kend = min(K, kbeg + split_len);
  const int nstep = (kend - kbeg + kBf16Step - 1) / kBf16Step;

  const float* arow[TM];
  float asub[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int row = row_base + 16 * t + r16;
    if (row < m || row >= arows) {
      arow[t] = R + (row < m ? row : 0) * ldr;
      asub[t] = row < m ? r0[row] : 0.0f;
    } else {
      arow[t] = Wf + static_cast<int64_t>(row - m) * ldw;
      asub[t] = 0.0f;
    }
  }
  // the B pieces this thread copies: piece c -> (plane, column, k-group),
  // k-group fastest so that 8 neighbouring threads read one 128-byte run;
  // pieces of the padding columns (and past CHUNKS) read column 0 and are
  // not stored
  const __bf16* bsrc[PER_THREAD];
  const float* wsrc[PER_THREAD];
  int bkg[PER_THREAD];
  bool bvalid[PER_THREAD];
#pragma unroll
  for (int i = 0; i < PER_THREAD; ++i) {
    const int c = tid + 256 * i;
    const int kg = c % (kBf16Step / 8), col = (c / (kBf16Step / 8)) % NCOL;
    const int pl = c / (NCOL * (kBf16Step / 8));
    bvalid[i] = c < CHUNKS && col < n;
    bkg[i] = 8 * kg;
    const int64_t cc = col < n ? col : 0;
    if constexpr (WF32)
      wsrc[i] = Wf + cc * ldw;
    else
      bsrc[i] = (PLANES == 2 && pl == 1 ? Bl : Bh) + cc * kpad;
  }
  auto load_b = [&](int k0, BReg (&reg)[PER_THREAD]) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int kk = k0 + bkg[i];
      const int kc = kk < kend ? kk : kbeg;
      if constexpr (WF32 && VEC) {
        const f32x4 x0 = *reinterpret_cast<const f32x4*>(wsrc[i] + kc);
        const f32x4 x1 = *reinterpret_cast<const f32x4*>(wsrc[i] + kc + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          reg[i][e] = x0[e];
          reg[i][4 + e] = x1[e];
        }
      } else if constexpr (WF32) {
#pragma unroll
        for (int e = 0; e < 8; ++e) reg[i][e] = wsrc[i][min(kc + e, K - 1)];
      } else {
        reg[i] = *reinterpret_cast<const bf16x8*>(bsrc[i] + kc);
      }
    }
  };
  // the padding columns' pieces hold zeros in both buffers from the start
  // and are never written again
#pragma unroll
  for (int i = 0; i < PER_THREAD; ++i) {
    const int c = tid + 256 * i;
    if (c < CHUNKS && !bvalid[i]) {
      const int kg = c % (kBf16Step / 8), col = (c / (kBf16Step / 8)) % NCOL;
#pragma unroll
      for (int pl = 0; pl < PLANES; ++pl) {
        if (WF32 || pl == c / (NCOL * (kBf16Step / 8))) {
          stage[0][pl][kg][col] = bf16x8{};
          stage[1][pl][kg][col] = bf16x8{};
        }
      }
    }
  }
  auto store_b = [&](int buf, const BReg (&reg)[PER_THREAD]) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int c = tid + 256 * i;
      if (bvalid[i]) {
        const int kg = c % (kBf16Step / 8), col = (c / (kBf16Step / 8)) % NCOL;
        if constexpr (WF32) {
          bf16x8 h, l;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            h[e] = static_cast<__bf16>(reg[i][e]);
            l[e] = static_cast<__bf16>(reg[i][e] - static_cast<float>(h[e]));
          }
          stage[buf][0][kg][col] = h;
          if constexpr (TERMS == 3) stage[buf][PLANES - 1][kg][col] = l;
        } else {
          const int pl = c / (NCOL * (kBf16Step / 8));
          stage[buf][pl][kg][col] = reg[i];
        }
      }
    }
  };
  // this lane's 8 raw A values of row tile t for the step at k0 (a group past
  // the slice reads the slice's first group); the r0 shift and the zeros past
  // kend are applied where they are used
  auto load_a = [&](int k0, float (&a)[TM][8]) {
    const int kl = k0 + 8 * kq;
    const int kc = kl < kend ? kl : kbeg;
    if constexpr (VEC) {
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const f32x4 x0 = *reinterpret_cast<const f32x4*>(arow[t] + kc);
        const f32x4 x1 = *reinterpret_cast<const f32x4*>(arow[t] + kc + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a[t][e] = x0[e];
          a[t][4 + e] = x1[e];
        }
      }
    } else {
      // one value per load, each clamped into the row
#pragma unroll
      for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) a[t][e] = arow[t][min(kc + e, K - 1)];
    }
  };

  f32x4 acc[TM][NT];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int tn = 0; tn < NT; ++tn) acc[t][tn] = f32x4{0, 0, 0, 0};

  // A(s) sits in ring slot s % D and is reloaded with A(s + D) once it has
  // been converted; B(s + 2) is fetched into buffer s % 2 at the start of
  // step s, and B(s + 1) (fetched at step s - 1) goes to LDS at its end
  if (nstep > 0) {  // uniform
    float a[D][TM][8];
    BReg breg[2][PER_THREAD];
    load_b(kbeg, breg[0]);
#pragma unroll
    for (int d = 0; d < D; ++d) load_a(kbeg + d * kBf16Step, a[d]);
    load_b(kbeg + kBf16Step, breg[1]);
    store_b(0, breg[0]);
    __syncthreads();
    // step at k0; LOADS: fetch B two and A kBf16Depth steps ahead (every
    // ring turn but the last), STORE: hand B of the next step to LDS
    auto step = [&](int k0, float (&as)[TM][8], BReg (&bnext)[PER_THREAD],
                    BReg (&bstore)[PER_THREAD], int buf, auto loads, auto store) {
      if constexpr (decltype(loads)::value) load_b(k0 + 2 * kBf16Step, bnext);
      const int kl = k0 + 8 * kq;
      bf16x8 ah[TM], al[TM];
      if (k0 + kBf16Step <= kend) {  // uniform: a whole step inside the slice
#pragma unroll
        for (int t = 0; t < TM; ++t)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float v = as[t][e] - asub[t];
            ah[t][e] = static_cast<__bf16>(v);
            if constexpr (TERMS == 3)
              al[t][e] = static_cast<__bf16>(v - static_cast<float>(ah[t][e]));
          }
      } else {
#pragma unroll
        for (int t = 0; t < TM; ++t)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float v = (kl + e < kend) ? as[t][e] - asub[t] : 0.0f;
            ah[t][e] = static_cast<__bf16>(v);
            if constexpr (TERMS == 3)
              al[t][e] = static_cast<__bf16>(v - static_cast<float>(ah[t][e]));
          }
      }
      if constexpr (decltype(loads)::value) load_a(k0 + D * kBf16Step, as);
#pragma unroll
      for (int tn = 0; tn < NT; ++tn) {
        const bf16x8 bh = stage[buf][0][kq][16 * tn + r16];
#pragma unroll
        for (int t = 0; t < TM; ++t)
          acc[t][tn] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[t], bh, acc[t][tn], 0, 0, 0);
        if constexpr (TERMS == 3) {
          const bf16x8 bl = stage[buf][PLANES - 1][kq][16 * tn + r16];
#pragma unroll
          for (int t = 0; t < TM; ++t) {
            acc[t][tn] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[t], bl, acc[t][tn], 0, 0, 0);
            acc[t][tn] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[t], bh, acc[t][tn], 0, 0, 0);
          }
        }
      }
      if constexpr (decltype(store)::value) store_b(buf ^ 1, bstore);
      __syncthreads();
    };
    // whole ring turns; the last one fetches nothing and stores only the B
    // of its own steps
    const int nturn = (nstep + D - 1) / D;
    for (int s = 0; s < (nturn - 1) * D; s += D) {
#pragma unroll
      for (int d = 0; d < D; ++d)
        step(kbeg + (s + d) * kBf16Step, a[d], breg[d & 1], breg[(d + 1) & 1], d & 1,
             std::true_type{}, std::true_type{});
    }
    static_for<0, D>([&](auto dc) {
      constexpr int d = decltype(dc)::value;
      step(kbeg + ((nturn - 1) * D + d) * kBf16Step, a[d], breg[d & 1], breg[(d + 1) & 1], d & 1,
           std::false_type{}, std::integral_constant<bool, (d + 1 < D)>{});
    });
  }
  float* out = part + static_cast<int64_t>(by) * arows * npad;
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row_base + 16 * t + 4 * kq + j;
      if (row < arows)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn) out[row * npad + 16 * tn + r16] = acc[t][tn][j];
    }
}

template <int TERMS, int NT, int TM, bool VEC>
__global__ void __launch_bounds__(256) contract_bf16_kernel(
    int m, int n, int K, const float* __restrict__ R, int64_t ldr, const float* __restrict__ r0,
    const float* __restrict__ Wf, int64_t ldw, int split_len, float* __restrict__ part,
    int npad, int arows) {
  contract_bf16_block<TERMS, NT, TM, VEC, true>(m, n, K, R, ldr, r0, nullptr, nullptr, 0, split_len,
                                                part, npad, blockIdx.x, blockIdx.y, Wf, ldw, arows);
}

// Batched S = (R - r0 1^T) W^T partials, BF16x3; tile = split * row_blocks + row block.
template <int NT>
__global__ void __launch_bounds__(256) batch_contract_bf16_kernel(const BatchInst* __restrict__ inst,
                                                                  BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    const int rb = (b.m + 64 * kBatchBf16RowTiles - 1) / (64 * kBatchBf16RowTiles);
    contract_bf16_block<3, NT, kBatchBf16RowTiles, true>(b.m, b.n, b.K, b.R, b.ldr, b.r0, b.Wh, b.Wl,
                                                    b.kpad, b.split_len, b.part, b.npad,
                                                    it.tile % rb, it.tile / rb);
    __syncthreads();
  }
}

template <int TERMS, bool VEC>
hipError_t bf16_dispatch(int nt, dim3 grid, hipStream_t st, int m, int n, int K, const float* R,
                         int64_t ldr, const float* r0, const float* W, int64_t ldw,
                         int split_len, float* part, int npad, int arows) {
#define GNM_BF_CASE(NT)                                                                        \
  case NT:                                                                                     \
    hipLaunchKernelGGL((contract_bf16_kernel<TERMS, NT, bf16_row_tiles(TERMS), VEC>), grid,      \
                       dim3(256), 0,                                                              \
                       st, m, n, K, R, ldr, r0, W, ldw, split_len, part, npad, arows);         \
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

#ifdef GNM_GEMM_PLAIN_UNIT
// The plain-BF16 contraction (one product per term), from its own unit.
hipError_t launch_contract_bf16_plain(int nt, dim3 grid, hipStream_t st, int m, int n, int K,
                                      const float* R, int64_t ldr, const float* r0, const float* W,
                                      int64_t ldw, int split_len, float* part, int npad,
                                      int arows, bool vec) {
  return vec ? bf16_dispatch<1, true>(nt, grid, st, m, n, K, R, ldr, r0, W, ldw, split_len, part,
                                      npad, arows)
             : bf16_dispatch<1, false>(nt, grid, st, m, n, K, R, ldr, r0, W, ldw, split_len, part,
                                       npad, arows);
}
#else
int contract_kw(size_t elem_size, int ncol) {
  const int nt = (ncol + 15) / 16;
  // the split epilogue parks 4 waves' tiles in LDS: stay within 64 KB
  return static_cast<size_t>(4) * 16 * (16 * nt + 1) * elem_size <= 65536 ? 4 : 1;
}

hipError_t launch_contract(const ContractArgs<float>& a, int nsplit, hipStream_t st) {
  return contract_typed(a, nsplit, st);
}
hipError_t launch_contract(const ContractArgs<double>& a, int nsplit, hipStream_t st) {
  return contract_typed(a, nsplit, st);
}

int batch_contract_row_blocks(int rows) { return (rows + 15) / 16; }
int batch_bf16_row_blocks(int m) {
  return (m + 64 * kBatchBf16RowTiles - 1) / (64 * kBatchBf16RowTiles);
}

hipError_t launch_batch_contract(int nt, const BatchInst* inst, const BatchLaunch& L,
                                 hipStream_t st) {
  if (L.count == 0) return hipSuccess;
#define GNM_BC_CASE(NT)                                                                          \
  case NT:                                                                                       \
    hipLaunchKernelGGL((batch_contract_kernel<NT>), dim3(L.blocks), dim3(256),                  \
                       (split_lds_bytes<float, NT>()), st, inst, L);                            \
    break;
  switch (nt) {
    GNM_BC_CASE(1) GNM_BC_CASE(2) GNM_BC_CASE(3) GNM_BC_CASE(4) GNM_BC_CASE(5) GNM_BC_CASE(6)
    GNM_BC_CASE(7) GNM_BC_CASE(8) GNM_BC_CASE(9) GNM_BC_CASE(10) GNM_BC_CASE(11) GNM_BC_CASE(12)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_BC_CASE
  return hipGetLastError();
}

hipError_t launch_batch_split_bf16(const BatchInst* inst, const BatchLaunch& L, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_split_bf16_kernel, dim3(L.blocks), dim3(256), 0, st, inst, L);
  return hipGetLastError();
}

hipError_t launch_batch_contract_bf16(int nt, const BatchInst* inst, const BatchLaunch& L,
                                      hipStream_t st) {
  if (L.count == 0) return hipSuccess;
#define GNM_BB_CASE(NT)                                                                          \
  case NT:                                                                                       \
    hipLaunchKernelGGL((batch_contract_bf16_kernel<NT>), dim3(L.blocks), dim3(256), 0, st, inst, L); \
    break;
  switch (nt) {
    GNM_BB_CASE(1) GNM_BB_CASE(2) GNM_BB_CASE(3) GNM_BB_CASE(4) GNM_BB_CASE(5) GNM_BB_CASE(6)
    GNM_BB_CASE(7) GNM_BB_CASE(8) GNM_BB_CASE(9) GNM_BB_CASE(10) GNM_BB_CASE(11) GNM_BB_CASE(12)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_BB_CASE
  return hipGetLastError();
}


hipError_t launch_contract_bf16(int terms, int m, int n, int K, const float* R, int64_t ldr,
                                const float* r0, const float* W, int64_t ldw, int nsplit,
                                int split_len, float* part, int npad, hipStream_t st,
                                bool with_gram) {
  const int arows = with_gram ? m + n : m;
  const int rt = bf16_row_tiles(terms);
  dim3 grid((arows + 64 * rt - 1) / (64 * rt), nsplit);
  const int nt = (n + 15) / 16;
  // 16-byte loads of whole 8-value groups: aligned rows of R and W, and K % 8
  // == 0 so that no group runs past the end of a row
  const bool vec = (ldr % 4 == 0) && (reinterpret_cast<uintptr_t>(R) % 16 == 0) &&
                   (ldw % 4 == 0) && (reinterpret_cast<uintptr_t>(W) % 16 == 0) && (K % 8 == 0);
  if (terms == 3)
    return vec ? bf16_dispatch<3, true>(nt, grid, st, m, n, K, R, ldr, r0, W, ldw, split_len, part,
                                        npad, arows)
               : bf16_dispatch<3, false>(nt, grid, st, m, n, K, R, ldr, r0, W, ldw, split_len, part,
                                         npad, arows);
  return launch_contract_bf16_plain(nt, grid, st, m, n, K, R, ldr, r0, W, ldw, split_len, part,
                                    npad, arows, vec);
}
#endif  // GNM_GEMM_PLAIN_UNIT

}  // namespace gnm
