// Batched rollout fused with the sample contraction of the LS Jacobian
// (Eqs. (1), (2), (4) and (10)): the residual rows never reach HBM.
//
// With antithetic pairs (W[:, s + K/2] = -W[:, s]) the nominal residual
// cancels from the contraction:
//   (R_s - r0) W_s^T + (R_s' - r0) W_s'^T = (R_s - R_s') W_s^T,  s' = s + K/2,
// so S = dR W^T = sum over the K/2 pairs of D_s W_s^T with D_s = R_s - R_s'.
// And since R_s = w .* (x_s - x_ref) row by row (w the square roots of 2 q
// and 2 r), D_s = w .* (x_s - x_s'): the reference cancels too and the row
// weight can be applied to the finished rows of S.
//
// Mapping (one work item = 128 antithetic pairs of one instance, 512
// threads):
//  * waves 0-3 roll out one sample per lane, the whole chain state in
//    registers: lanes 0-31 of a wave the samples s, lanes 32-63 their
//    partners s' (so one lane-half swap, v_permlane32_swap, gives every lane
//    its pair's difference); after each step they write the pair
//    differences of the step's 4M + 2 rows into a double-buffered LDS tile
//    [row][pair] and meet the other waves at a barrier;
//  * waves 4-7 contract the tile of the previous step with the block's W
//    columns (staged once per item in LDS as bf16 hi/lo planes) on the BF16
//    MFMA, three products per term (hi hi, hi lo, lo hi: FP32-level error),
//    scale the rows by their weights and store them as this item's partial
//    sum of S (one partial per 128 pairs; a later step adds the partials).
// One rollout wave and one contraction wave share each SIMD, so the RK4
// arithmetic and the MFMA work overlap.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace gnm {
namespace {

using f32x4 = float __attribute__((ext_vector_type(4)));
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));

constexpr int kPairs = kFusedPairs;         // antithetic pairs per work item
constexpr int kFusedThreads = 512;          // 4 rollout waves + 4 contraction waves
constexpr int kDLd = kPairs + 4;            // LDS row stride of the difference tile (floats)
constexpr int kWLd = kPairs + 8;            // LDS row stride of a W plane (bf16)
constexpr int kMaxNpad = 160;               // n = 2N <= 160 (N <= 80)
constexpr int kColSlots = 3;                // 16-column tiles per contraction wave: ceil(10 / 4)

// Chain constants shared by every instance of a batch.
struct FusedChain {
  float dt, k_lin, k_cub, inv_mass;
};

template <int M>
struct FusedShape {
  static constexpr int kRows = 4 * M + 2;                // residual rows per step
  static constexpr int kRowTiles = (kRows + 15) / 16;
};

// One RK4 stage for a sample held in one lane.  The stage input is
// (p, v) + c (kp, kv / mass) with (kp, kv) the previous stage's derivative
// (zero before the first stage), cim = c / mass; its derivative overwrites
// (kp, kv) and is added to the running sums with weight wgt.  The chain's
// right-hand side: link tension T_i = (k_lin + k_cub |d_i|^2) d_i with
// d_i = P_i - P_{i-1} (P_{-1} the anchor at the origin); a free mass
// accelerates by (T_{i+1} - T_i) / mass, and kv holds the tension difference
// itself (every free mass has the same mass, which the caller folds into its
// constants: no multiply per mass and stage); the end mass (i = M - 1) moves
// with its velocity slot, which holds the commanded velocity, and does not
// accelerate.  The masses are streamed in order, so only two tensions are
// live at a time.
template <int M>
__device__ __forceinline__ void chain_stage_lane(const float (&px)[M], const float (&py)[M],
                                                 const float (&vx)[M], const float (&vy)[M],
                                                 float (&kpx)[M], float (&kpy)[M],
                                                 float (&kvx)[M], float (&kvy)[M], float (&spx)[M],
                                                 float (&spy)[M], float (&svx)[M],
                                                 float (&svy)[M], float c, float cim, float wgt,
                                                 float k_lin, float k_cub) {
  float qx = 0.0f, qy = 0.0f;  // stage position of the previous mass (the anchor first)
  float tpx = 0.0f, tpy = 0.0f;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const float Px = px[i] + c * kpx[i], Py = py[i] + c * kpy[i];
    const float dx = Px - qx, dy = Py - qy;
    const float s = k_lin + k_cub * (dx * dx + dy * dy);
    const float tx = s * dx, ty = s * dy;
    if (i > 0) {  // mass i - 1 is complete: it needed T_i
      const int j = i - 1;
      const float nvx = tx - tpx, nvy = ty - tpy;
      kpx[j] = vx[j] + cim * kvx[j];
      kpy[j] = vy[j] + cim * kvy[j];
      kvx[j] = nvx;
      kvy[j] = nvy;
      spx[j] += wgt * kpx[j];
      spy[j] += wgt * kpy[j];
      svx[j] += wgt * kvx[j];
      svy[j] += wgt * kvy[j];
    }
    qx = Px;
    qy = Py;
    tpx = tx;
    tpy = ty;
  }
  constexpr int j = M - 1;  // the end mass: no acceleration
  kpx[j] = vx[j] + cim * kvx[j];
  kpy[j] = vy[j] + cim * kvy[j];
  kvx[j] = 0.0f;
  kvy[j] = 0.0f;
  spx[j] += wgt * kpx[j];
  spy[j] += wgt * kpy[j];
}

// One classical RK4 step of length h with the control held (the end mass's
// velocity slot is set to the control before the step).
template <int M>
__device__ __forceinline__ void chain_rk4_lane(float (&px)[M], float (&py)[M], float (&vx)[M],
                                               float (&vy)[M], float u0, float u1, float h,
                                               float k_lin, float k_cub, float im) {
  vx[M - 1] = u0;
  vy[M - 1] = u1;
  const float hh = 0.5f * h, h6 = h / 6.0f;
  float kpx[M], kpy[M], kvx[M], kvy[M], spx[M], spy[M], svx[M], svy[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    kpx[i] = kpy[i] = kvx[i] = kvy[i] = 0.0f;
    spx[i] = spy[i] = svx[i] = svy[i] = 0.0f;
  }
  chain_stage_lane<M>(px, py, vx, vy, kpx, kpy, kvx, kvy, spx, spy, svx, svy, 0.0f, 0.0f, 1.0f,
                      k_lin, k_cub);
  chain_stage_lane<M>(px, py, vx, vy, kpx, kpy, kvx, kvy, spx, spy, svx, svy, hh, hh * im, 2.0f,
                      k_lin, k_cub);
  chain_stage_lane<M>(px, py, vx, vy, kpx, kpy, kvx, kvy, spx, spy, svx, svy, hh, hh * im, 2.0f,
                      k_lin, k_cub);
  chain_stage_lane<M>(px, py, vx, vy, kpx, kpy, kvx, kvy, spx, spy, svx, svy, h, h * im, 1.0f,
                      k_lin, k_cub);
  const float h6im = h6 * im;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    px[i] += h6 * spx[i];
    py[i] += h6 * spy[i];
    vx[i] += h6im * svx[i];
    vy[i] += h6im * svy[i];
  }
}

// Pair differences of an (x, y) value held by every lane: lanes 0-31 (the
// samples s) get x(s) - x(s'), lanes 32-63 (the partners s') get
// y(s) - y(s').  v_permlane32_swap exchanges the upper half of its first
// operand with the lower half of its second, which leaves
// {x_lo, y_lo} = (s values) in the first and {x_hi, y_hi} = (s' values) in
// the second, each lane holding the component its half writes.
__device__ __forceinline__ float pair_diff_xy(float x, float y) {
  const auto h = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(int, x),
                                                  __builtin_bit_cast(int, y), false, false);
  return __builtin_bit_cast(float, static_cast<int>(h[0])) -
         __builtin_bit_cast(float, static_cast<int>(h[1]));
}

// One step of a rollout lane: RK4, then the pair differences of the step's
// rows into dbuf[k & 1] and the barrier that hands the tile over.  Lanes
// 0-31 write the even rows (x components and u_0), lanes 32-63 the odd rows
// (y components and u_1).  Lanes past the item's last pair roll out a valid
// sample and write finite differences; their W columns are zero, so they
// add nothing to S.
template <int M>
__device__ __forceinline__ void fused_rollout_step(float (&px)[M], float (&py)[M], float (&vx)[M],
                                                   float (&vy)[M], float u0, float u1,
                                                   const FusedChain& cd, int k, int half, int p,
                                                   float* dbuf) {
  constexpr int R = FusedShape<M>::kRows;
  constexpr int DB = R * kDLd;  // floats per buffer
  chain_rk4_lane<M>(px, py, vx, vy, u0, u1, cd.dt, cd.k_lin, cd.k_cub, cd.inv_mass);
  float* t = dbuf + (k & 1) * DB + p;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    t[(2 * i + half) * kDLd] = pair_diff_xy(px[i], py[i]);
    t[(2 * M + 2 * i + half) * kDLd] = pair_diff_xy(vx[i], vy[i]);
  }
  t[(4 * M + half) * kDLd] = pair_diff_xy(u0, u1);
  __syncthreads();  // step k's tile is complete
}

// Rollout waves: the item's pairs, one sample per lane, and the pair
// differences of every step into dbuf[k & 1].  Lanes 0-31 write the even rows
// (x components and u_0), lanes 32-63 the odd rows (y components and u_1).
// Perturbation loads run ahead of their use: a global load takes about as
// long as a few RK4 steps of a small chain, a step of a long chain covers
// most of it (and its registers are scarce).
template <int M>
constexpr int w_ahead() {
  return M <= 10 ? 4 : 2;
}

template <int M>
__device__ __forceinline__ void fused_rollout_role(const BatchInst& b, const FusedChain& cd,
                                                   int s0, float* dbuf, const float* ush, int lane,
                                                   int wave) {
  constexpr int WA = w_ahead<M>();
  const int half = lane >> 5;
  const int p = wave * 32 + (lane & 31);  // pair within the item
  const int Kh = b.K / 2;
  const int s = s0 + p < Kh ? s0 + p : 0;
  const int col = half ? s + Kh : s;
  float px[M], py[M], vx[M], vy[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    px[i] = b.x0[2 * i];
    py[i] = b.x0[2 * i + 1];
    vx[i] = b.x0[2 * M + 2 * i];
    vy[i] = b.x0[2 * M + 2 * i + 1];
  }
  const int N = b.N;
  const int64_t ldw = b.ldw;
  const float* __restrict__ Wc = b.W + col;
  // perturbations of steps k .. k + WA - 1 in flight (a ring indexed by
  // k mod WA, unrolled so that the index is a constant)
  float wq0[WA], wq1[WA];
#pragma unroll
  for (int t = 0; t < WA; ++t) {
    const int kk = t < N ? t : 0;
    wq0[t] = Wc[(2 * kk) * ldw];
    wq1[t] = Wc[(2 * kk + 1) * ldw];
  }
  for (int k0 = 0; k0 < N; k0 += WA) {
#pragma unroll
    for (int t = 0; t < WA; ++t) {
      const int k = k0 + t;
      if (k >= N) break;  // uniform
      const float u0 = ush[2 * k] + wq0[t], u1 = ush[2 * k + 1] + wq1[t];
      const int kn = k + WA < N ? k + WA : k;
      wq0[t] = Wc[(2 * kn) * ldw];
      wq1[t] = Wc[(2 * kn + 1) * ldw];
      fused_rollout_step<M>(px, py, vx, vy, u0, u1, cd, k, half, p, dbuf);
    }
  }
}

// Contraction waves: for every step, S_k (R rows x n) of this item's pairs,
// from the tile of that step and the staged W planes; wave mw takes the
// column tiles mw, mw + 4, mw + 8.
template <int M>
__device__ __forceinline__ void fused_contract_role(const BatchInst& b, int item, const float* dbuf,
                                                    const __bf16* wh, const __bf16* wl,
                                                    const float* wrow, int lane, int mw) {
  constexpr int R = FusedShape<M>::kRows;
  constexpr int RT = FusedShape<M>::kRowTiles;
  constexpr int DB = R * kDLd;
  const int ct = b.npad / 16;
  const int l16 = lane & 15, q = lane >> 4;
  float* __restrict__ part = b.part + static_cast<int64_t>(item) * (b.m + b.grows) * b.npad;
  // Row tile tr of this item's G = W W^T, 2 sum over its pairs w_s w_s^T
  // (each pair's partner is -w_s), from the same bf16 planes (BF16x3), into
  // the rows below S of the item's partial: the tiles (tr, tc) with tc <= tr,
  // each also stored transposed, so G is exactly symmetric.  One row tile
  // per step, so the work spreads over the first steps instead of delaying
  // the first.
  auto gram_row_tile = [&](int tr) {
    f32x4 acc[kColSlots];
#pragma unroll
    for (int c = 0; c < kColSlots; ++c) acc[c] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kPairs / 32; ++kk) {
      const int k0 = 32 * kk + 8 * q;
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(wh + (16 * tr + l16) * kWLd + k0);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(wl + (16 * tr + l16) * kWLd + k0);
#pragma unroll
      for (int c = 0; c < kColSlots; ++c) {
        const int tc = mw + 4 * c;
        if (tc <= tr) {  // uniform
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(wh + (16 * tc + l16) * kWLd + k0);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(wl + (16 * tc + l16) * kWLd + k0);
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[c], 0, 0, 0);
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[c], 0, 0, 0);
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[c], 0, 0, 0);
        }
      }
    }
    float* gdst = part + static_cast<int64_t>(b.m) * b.npad;
#pragma unroll
    for (int c = 0; c < kColSlots; ++c) {
      const int tc = mw + 4 * c;
      if (tc <= tr) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 16 * tr + 4 * q + e, col = 16 * tc + l16;
          const float v = 2.0f * acc[c][e];
          if (row < b.n) gdst[static_cast<int64_t>(row) * b.npad + col] = v;
          if (tc < tr && col < b.n) gdst[static_cast<int64_t>(col) * b.npad + row] = v;
        }
      }
    }
  };
  for (int k = 0; k < b.N; ++k) {
    __syncthreads();  // step k's tile is complete
    const float* t = dbuf + (k & 1) * DB;
    f32x4 acc[RT][kColSlots];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < kColSlots; ++c) acc[r][c] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kPairs / 32; ++kk) {
      const int k0 = 32 * kk + 8 * q;
      bf16x8 bh[kColSlots], bl[kColSlots];
#pragma unroll
      for (int c = 0; c < kColSlots; ++c) {
        const int tc = mw + 4 * c;
        const int row = (tc < ct ? tc : 0) * 16 + l16;  // clamped: unused slots read tile 0
        bh[c] = *reinterpret_cast<const bf16x8*>(wh + row * kWLd + k0);
        bl[c] = *reinterpret_cast<const bf16x8*>(wl + row * kWLd + k0);
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int row = 16 * r + l16;
        const bool in = row < R;  // the last row tile overhangs the tile's rows
        const float* src = t + (in ? row : 0) * kDLd + k0;
        const f32x4 v0 = *reinterpret_cast<const f32x4*>(src);
        const f32x4 v1 = *reinterpret_cast<const f32x4*>(src + 4);
        bf16x8 ah, al;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float v = in ? (e < 4 ? v0[e] : v1[e - 4]) : 0.0f;
          ah[e] = static_cast<__bf16>(v);
          al[e] = static_cast<__bf16>(v - static_cast<float>(ah[e]));
        }
#pragma unroll
        for (int c = 0; c < kColSlots; ++c) {
          if (mw + 4 * c < ct) {  // uniform
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[r][c], 0, 0, 0);
          }
        }
      }
    }
    // rows of step k: weight each row and store the item's partial sum
    float* dst = part + static_cast<int64_t>(k) * R * b.npad;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < kColSlots; ++c) {
        const int tc = mw + 4 * c;
        if (tc < ct) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = 16 * r + 4 * q + e;
            if (row < R) dst[static_cast<int64_t>(row) * b.npad + 16 * tc + l16] = wrow[row] * acc[r][c][e];
          }
        }
      }
    if (b.grows > 0 && k < ct) gram_row_tile(k);
  }
  if (b.grows > 0)
    for (int tr = b.N; tr < ct; ++tr) gram_row_tile(tr);
}

// LDS of a block, sized for the longest chain (M = 16): the difference tile
// (two buffers of 4 M + 2 rows), the W planes, the row weights and U.
struct FusedLds {
  float dbuf[2 * FusedShape<16>::kRows * kDLd];
  __bf16 wplanes[2 * kMaxNpad * kWLd];
  float wrow[FusedShape<16>::kRows];
  float ush[kMaxNpad];
};

// Item = (instance, pair block j): pairs 128 j .. 128 j + 127 of the K/2.
// Not inlined: each chain length gets its own register allocation (inlined
// into one kernel, the fourteen bodies spill).
template <int M>
__device__ __attribute__((noinline)) void fused_item(const BatchInst& b, int tile, const FusedChain& cd,
                                           FusedLds& S, int lane, int wave) {
  constexpr int R = FusedShape<M>::kRows;
  __bf16* wh = S.wplanes;
  __bf16* wl = S.wplanes + kMaxNpad * kWLd;
  const int s0 = kPairs * tile;
  const int Kh = b.K / 2;
  // the block's W columns (the first member of each pair) as bf16 hi/lo
  // planes [row][pair], zero beyond n rows and K/2 pairs; row weights; U
  for (int e = threadIdx.x; e < b.npad * (kPairs / 8); e += kFusedThreads) {
    const int row = e / (kPairs / 8), c8 = 8 * (e % (kPairs / 8));
    bf16x8 h, l;
    if (row < b.n && s0 + c8 + 8 <= Kh) {
      h = *reinterpret_cast<const bf16x8*>(b.Wh + static_cast<int64_t>(row) * b.kpad + s0 + c8);
      l = *reinterpret_cast<const bf16x8*>(b.Wl + static_cast<int64_t>(row) * b.kpad + s0 + c8);
    } else {
#pragma unroll
      for (int x = 0; x < 8; ++x) {
        const bool ok = row < b.n && s0 + c8 + x < Kh;
        const int64_t o = static_cast<int64_t>(ok ? row : 0) * b.kpad + (ok ? s0 + c8 + x : 0);
        h[x] = ok ? b.Wh[o] : __bf16(0.0f);
        l[x] = ok ? b.Wl[o] : __bf16(0.0f);
      }
    }
    *reinterpret_cast<bf16x8*>(wh + row * kWLd + c8) = h;
    *reinterpret_cast<bf16x8*>(wl + row * kWLd + c8) = l;
  }
  for (int j = threadIdx.x; j < R; j += kFusedThreads)
    S.wrow[j] = __builtin_sqrtf(2.0f * (j < 4 * M ? b.q[j] : b.r[j - 4 * M]));
  for (int j = threadIdx.x; j < b.n; j += kFusedThreads) S.ush[j] = b.U[j];
  __syncthreads();
  if (wave < 4)
    fused_rollout_role<M>(b, cd, s0, S.dbuf, S.ush, lane, wave);
  else
    fused_contract_role<M>(b, tile, S.dbuf, wh, wl, S.wrow, lane, wave - 4);
  __syncthreads();  // the next item restages the W planes and the tile
}

// One persistent launch for every chain length: the items of all instances,
// longest first, each dispatched to the code of its M, so that blocks stay
// busy until the whole batch is done.
__global__ void __launch_bounds__(kFusedThreads) batch_fused_kernel(
    const BatchInst* __restrict__ inst, BatchLaunch L, FusedChain cd) {
  __shared__ __attribute__((aligned(16))) FusedLds S;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    switch (b.M) {  // uniform
#define GNM_FUSED_CASE(MM) \
  case MM:                 \
    fused_item<MM>(b, it.tile, cd, S, lane, wave); \
    break;
      GNM_FUSED_CASE(3) GNM_FUSED_CASE(4) GNM_FUSED_CASE(5) GNM_FUSED_CASE(6) GNM_FUSED_CASE(7)
      GNM_FUSED_CASE(8) GNM_FUSED_CASE(9) GNM_FUSED_CASE(10) GNM_FUSED_CASE(11)
      GNM_FUSED_CASE(12) GNM_FUSED_CASE(13) GNM_FUSED_CASE(14) GNM_FUSED_CASE(15)
      GNM_FUSED_CASE(16)
#undef GNM_FUSED_CASE
      default:
        break;  // 3 <= M <= 16 is checked when the batch is prepared
    }
  }
}

}  // namespace

hipError_t launch_batch_fused(const BatchInst* inst, const BatchLaunch& L,
                              const gnmppi_problem& shared, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  const FusedChain cd{static_cast<float>(shared.dt), static_cast<float>(shared.k_lin),
                      static_cast<float>(shared.k_cub), static_cast<float>(1.0 / shared.mass)};
  hipLaunchKernelGGL(batch_fused_kernel, dim3(L.blocks), dim3(kFusedThreads), 0, st, inst, L, cd);
  return hipGetLastError();
}

}  // namespace gnm
