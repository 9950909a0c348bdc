// Single-shooting rollouts with residuals and costs (Eqs. (1), (2), (4)) and
// the parallel line search of Eqs. (14)-(15).
//
// Mapping.  Double integrator: one lane per sample, the whole state in
// registers.  Chain: a group of G lanes (G = next power of two >= M, G <= 16)
// per sample, lane i holding mass i's position and velocity.  The spring
// force needs the neighbouring masses: lane i reads p_{i-1} and T_{i+1} from
// the adjacent lanes with one DPP row shift each (no LDS, no barrier), so an
// RK4 step costs about 100 VALU instructions per lane instead of ~1000 for a
// lane holding all 64 state entries, and the sequential horizon loop -- the
// latency that bounds a single MPC instance -- shrinks accordingly.
//
// Residual rows are stored sample-fastest (row i of column s at i*ldr + s).
// The chain kernel stages each step's rows in LDS and writes every row of
// the block as one contiguous segment; the double-integrator kernel's lanes
// already write consecutive columns.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "philox.hpp"

namespace gnm {
namespace {

// Threads per block of the batch rollout kernels.  Loops stride by this
// constant rather than blockDim.x: reading blockDim.x inside a loop costs a
// load of the dispatch packet, and its wait would also drain every store the
// rollout has in flight.
constexpr int kBlock = 256;

template <typename T>
struct ChainDev {
  int M;
  T dt, k_lin, k_cub, inv_mass;
};

// Controls are read in two parts so that a rollout can prefetch the raw
// loads several steps ahead and combine them only when the step runs:
// load(idx) returns {a, b}, value(a, b) the control entry.
//
// Perturbed sample s >= 0 (or the nominal, s < 0): U[idx] + W[idx, s].  The
// W load is unconditional (the nominal reads column 0 and masks it out), so
// no lane waits on it inside a divergent branch.
template <typename T>
struct CtrlPerturbed {
  const T* __restrict__ U;
  const T* __restrict__ W;  // may be null: every column uses U
  int64_t ldw;
  int s;
  __device__ __forceinline__ void load(int idx, T& a, T& b) const {
    a = U[idx];
    b = W ? W[idx * ldw + (s >= 0 ? s : 0)] : T(0);
  }
  __device__ __forceinline__ T value(T a, T b) const { return s >= 0 ? a + b : a; }
  __device__ __forceinline__ T operator()(int idx) const {
    T a, b;
    load(idx, a, b);
    return value(a, b);
  }
};

// Line-search candidate U + alpha dU.
template <typename T>
struct CtrlLine {
  const T* U;  // updated in place by the same kernel after a barrier
  const T* __restrict__ dU;
  T alpha;
  __device__ __forceinline__ void load(int idx, T& a, T& b) const {
    a = U[idx];
    b = dU[idx];
  }
  __device__ __forceinline__ T value(T a, T b) const { return a + alpha * b; }
  __device__ __forceinline__ T operator()(int idx) const { return U[idx] + alpha * dU[idx]; }
};

// Controls staged in LDS: ctl[idx * stride + slot].  The batch rollout
// stages U + W[:, s] for the block's samples (slot = sample in block), the
// line search stages U and dU once (stride 1) and combines them per step.
template <typename T>
struct CtrlStaged {
  const T* ctl;
  int stride, slot;
  __device__ __forceinline__ T operator()(int idx) const { return ctl[idx * stride + slot]; }
};

template <typename T>
struct CtrlLineStaged {
  const T* Us;
  const T* dUs;
  T alpha;
  __device__ __forceinline__ T operator()(int idx) const { return Us[idx] + alpha * dUs[idx]; }
};

// ---- chain ---------------------------------------------------------------

// a - b, never fused with a product that produces b: keeps the neighbour
// tension's row shift foldable into the subtraction (v_sub_f32 with a DPP
// operand) instead of a separate DPP move feeding a fused multiply-add.
template <typename T>
__device__ __forceinline__ T sub_unfused(T a, T b) {
#pragma clang fp contract(off)
  return a - b;
}

// Right-hand side for mass i (lane i of the group): dp = v, and the tension
// difference f = T_{i+1} - T_i, whose product with the lane's inverse mass is
// dv; the caller folds the inverse mass into its step constants, so the
// stages carry f and no multiply per stage.  The end mass moves with the
// commanded velocity: its lane enters every step with v = u and inverse mass
// 0, so the stages keep v = u and dp = v is the commanded velocity with no
// per-stage select.  With G < 16 the last lane of a group reads T_{i+1} from
// the first lane of the next sample's group, which may be infinite if that
// sample diverged; inf * 0 would carry a NaN into this sample, so lanes
// without a free mass select f = 0 there (a select, so finite results are
// unchanged bit for bit).
template <typename T, int G>
__device__ __forceinline__ void chain_rhs(T px, T py, T vx, T vy, const ChainDev<T>& cd, bool first,
                                          bool free_mass, T& dpx, T& dpy, T& fx, T& fy) {
  T qx = 0, qy = 0;
  if constexpr (G > 1) {
    qx = dpp_move<kDppRowShr1>(px);
    qy = dpp_move<kDppRowShr1>(py);
  }
  // link 1 is attached to the fixed anchor at the origin; with G = 16 the
  // group is a whole 16-lane row and the row shift already brings in zero
  if (G < 16 && first) {
    qx = 0;
    qy = 0;
  }
  const T dx = px - qx, dy = py - qy;
  const T s = cd.k_lin + cd.k_cub * (dx * dx + dy * dy);
  const T tx = s * dx, ty = s * dy;
  T nx = 0, ny = 0;
  if constexpr (G > 1) {
    nx = dpp_move<kDppRowShl1>(tx);
    ny = dpp_move<kDppRowShl1>(ty);
  }
  dpx = vx;
  dpy = vy;
  fx = sub_unfused(nx, tx);
  fy = sub_unfused(ny, ty);
  if constexpr (G < 16) {
    fx = free_mass ? fx : T(0);
    fy = free_mass ? fy : T(0);
  }
}

// Residual sinks of the chain rollout.  NoSink keeps only the cost.
struct NoSink {
  template <typename T>
  __device__ __forceinline__ void step(int, int, bool, bool, T, T, T, T, T, T) {}
};

// One sample's residual rows as a contiguous vector (row k (4M + 2) + ... of
// step k, the row order of R); rc == nullptr stores nothing.
template <typename T>
struct VectorSink {
  T* rc;
  int M;
  __device__ __forceinline__ void step(int k, int i, bool has_mass, bool first, T e0, T e1, T e2,
                                       T e3, T f0, T f1) {
    if (rc == nullptr) return;
    T* t = rc + k * (4 * M + 2);
    if (has_mass) {
      t[2 * i] = e0;
      t[2 * i + 1] = e1;
      t[2 * M + 2 * i] = e2;
      t[2 * M + 2 * i + 1] = e3;
    }
    if (first) {
      t[4 * M] = f0;
      t[4 * M + 1] = f1;
    }
  }
};

// Stores the first nfr rows of one residual tile t (rows base .. base + nfr
// of R, the columns col0 .. col0 + kSpb of the block) as contiguous row
// segments of the sample-fastest R (or into r0 for the nominal column K),
// four samples per store; tid in [0, kBlock) numbers the storing threads.
// Column K and the columns left of it in a partial last chunk go one row per
// thread; the threads that store column K also add its squares to csum, so
// the nominal cost needs no cost terms in the rollout itself.
template <typename T, int kSpb>
__device__ __forceinline__ void drain_tile(const T (*t)[kSpb + 1], int nfr, int64_t base, int tid,
                                           T* __restrict__ R, int64_t ldr, T* __restrict__ r0,
                                           int K, int col0, bool vec, T& csum) {
  constexpr int kVec = 4;                 // samples per vector store
  constexpr int kChunks = kSpb / kVec;    // vector stores per row
  static_assert(kSpb % kVec == 0 && kBlock % kChunks == 0, "chunking of a row");
  if (vec) {
    // whole 4-sample chunks left of column K: one vector store each
    using V = T __attribute__((ext_vector_type(kVec)));
    const int nvec = min(kChunks, max(0, (K - col0) / kVec));  // uniform
    // a thread keeps one 4-sample chunk of every (kBlock / kChunks)-th row,
    // so its LDS and HBM addresses advance by constant steps (the storing
    // waves share their SIMDs with the rollout waves: few instructions per
    // store)
    const int ch = tid % kChunks, sv = ch * kVec;
    if (ch < nvec) {
      constexpr int kRowStep = kBlock / kChunks;
      int fr = tid / kChunks;
      const T* src = &t[fr][sv];
      T* dst = R + (base + fr) * ldr + col0 + sv;
      const int64_t dstep = static_cast<int64_t>(kRowStep) * ldr;
      for (; fr < nfr; fr += kRowStep) {
        *reinterpret_cast<V*>(dst) = V{src[0], src[1], src[2], src[3]};
        src += kRowStep * (kSpb + 1);
        dst += dstep;
      }
    }
    // the block that holds column K: its last R columns one row per thread
    // (the bounds are uniform, so the stores need no divergent branches)
    const int ctail = col0 + nvec * kVec, cend = min(col0 + kSpb, K);
    if (ctail < cend)
      for (int fr = tid; fr < nfr; fr += kBlock)
        for (int c = ctail; c < cend; ++c) R[(base + fr) * ldr + c] = t[fr][c - col0];
  } else if (R) {
    for (int idx = tid; idx < nfr * kSpb; idx += kBlock) {
      const int fr = idx / kSpb, sc = idx % kSpb;
      if (col0 + sc < K) R[(base + fr) * ldr + col0 + sc] = t[fr][sc];
    }
  }
  // the nominal column, one row per thread whatever the layout of R (so c0
  // sums the same terms in the same order)
  if (col0 <= K && K < col0 + kSpb) {
    for (int fr = tid; fr < nfr; fr += kBlock) {
      const T v = t[fr][K - col0];
      if (r0) r0[base + fr] = v;
      csum += v * v;
    }
  }
}

// Residual tile of the block's samples in LDS, double-buffered: step j of a
// flush occupies rows j (4 M + 2) .., so the tile's rows are consecutive rows
// of R.  Row stride kSpb + 1: the G lanes of a sample write rows 2i of one
// column, which a stride of kSpb would put in a single LDS bank.
template <typename T, int G, int F>
struct ResidualTile {
  static constexpr int kSpb = kBlock / G;        // samples per block
  static constexpr int kRows = 4 * G + 2;        // >= rows per step (4 M + 2)
  static constexpr int kLd = kSpb + 1;
  using Buf = T[F * kRows][kLd];
  __device__ __forceinline__ static void put(Buf& b, int k, int M, int i, int grp, bool has_mass,
                                             bool first, T e0, T e1, T e2, T e3, T f0, T f1) {
    const int rows = 4 * M + 2;
    T (*t)[kLd] = b + (k % F) * rows;
    if (has_mass) {
      t[2 * i][grp] = e0;
      t[2 * i + 1][grp] = e1;
      t[2 * M + 2 * i][grp] = e2;
      t[2 * M + 2 * i + 1][grp] = e3;
    }
    if (first) {
      t[4 * M][grp] = f0;
      t[4 * M + 1][grp] = f1;
    }
  }
};

// StagedSink: the rollout threads write each step's rows into the tile and
// every F steps (and at the last step) store them themselves after a
// barrier (all threads of the block must call it).
template <typename T, int G, int F>
struct StagedSink {
  using Tile = ResidualTile<T, G, F>;
  static constexpr int kSpb = Tile::kSpb;
  static constexpr int kRows = Tile::kRows;
  static constexpr int kLd = Tile::kLd;
  T (*tile)[F * kRows][kLd];                     // [2][F kRows][kLd] in LDS
  T* R;
  int64_t ldr;
  T* r0;
  int K, col0, M, grp, N;
  bool vec;    // rows of R start 4-element aligned (uniform)
  T csum = 0;  // this thread's share of ||r||^2 of column K (the nominal)
  __device__ __forceinline__ void step(int k, int i, bool has_mass, bool first, T e0, T e1, T e2,
                                       T e3, T f0, T f1) {
    const int buf = (k / F) & 1, j = k % F;
    Tile::put(tile[buf], k, M, i, grp, has_mass, first, e0, e1, e2, e3, f0, f1);
    if (j != F - 1 && k != N - 1) return;  // uniform: flush every F steps and at the end
    __syncthreads();
    const int rows = 4 * M + 2;
    drain_tile<T, kSpb>(tile[buf], (j + 1) * rows, static_cast<int64_t>(k - j) * rows,
                        threadIdx.x, R, ldr, r0, K, col0, vec, csum);
  }
};

// TileSink: the rollout threads of a split block only fill the tile; at
// every F-th step (and the last) they meet the storing waves at a barrier
// and go on with the other buffer while those drain this one.
template <typename T, int G, int F>
struct TileSink {
  using Tile = ResidualTile<T, G, F>;
  T (*tile)[F * Tile::kRows][Tile::kLd];
  int M, grp, N;
  __device__ __forceinline__ void step(int k, int i, bool has_mass, bool first, T e0, T e1, T e2,
                                       T e3, T f0, T f1) {
    Tile::put(tile[(k / F) & 1], k, M, i, grp, has_mass, first, e0, e1, e2, e3, f0, f1);
    if (k % F == F - 1 || k == N - 1) __syncthreads();  // uniform
  }
};

// Steps per flush of StagedSink: about 24 KB of LDS per buffer.
template <typename T, int G>
constexpr int staged_flush_steps() {
  constexpr int per_step = (4 * G + 2) * (kBlock / G + 1) * static_cast<int>(sizeof(T));
  constexpr int f = 24576 / per_step;
  return f < 1 ? 1 : (f > 8 ? 8 : f);
}

// Rolls out one sample on the G lanes of its group and returns the group's
// cost 1/2 ||r||^2 (identical in every lane of the group; 0 without COST,
// which skips the cost terms).  All lanes of the wave must call this
// together (the DPP shifts read neighbouring lanes).
template <typename T, int G, bool COST, bool AHEAD = false, class Ctrl, class Sink>
__device__ __forceinline__ T chain_rollout(const ChainDev<T>& cd, int N,
                                           const T* __restrict__ x0, const T* __restrict__ q,
                                           const T* __restrict__ r, const T* __restrict__ xref,
                                           const Ctrl& ctrl, Sink& sink) {
  const int i = threadIdx.x & (G - 1);
  const int M = cd.M;
  const bool has_mass = i < M;
  const bool free_mass = i < M - 1;
  const bool first = i == 0;
  const int ii = has_mass ? i : 0;
  T px = has_mass ? x0[2 * ii] : T(0);
  T py = has_mass ? x0[2 * ii + 1] : T(0);
  T vx = has_mass ? x0[2 * M + 2 * ii] : T(0);
  T vy = has_mass ? x0[2 * M + 2 * ii + 1] : T(0);
  const T wpx = dsqrt(T(2) * q[2 * ii]), wpy = dsqrt(T(2) * q[2 * ii + 1]);
  const T wvx = dsqrt(T(2) * q[2 * M + 2 * ii]), wvy = dsqrt(T(2) * q[2 * M + 2 * ii + 1]);
  // residual w (x - x_ref) as one fused multiply-add: w x + (-w x_ref)
  const T cpx = -wpx * xref[2 * ii], cpy = -wpy * xref[2 * ii + 1];
  const T cvx = -wvx * xref[2 * M + 2 * ii], cvy = -wvy * xref[2 * M + 2 * ii + 1];
  const T wu0 = dsqrt(T(2) * r[0]), wu1 = dsqrt(T(2) * r[1]);
  const T h = cd.dt, hh = T(0.5) * cd.dt, h6 = cd.dt / T(6);
  // the step constants of the velocity times the lane's inverse mass (0 for
  // the end mass and the padding lanes): the stages carry the tension
  // differences f, and dv = f / mass enters only through these
  const T im = free_mass ? cd.inv_mass : T(0);
  const T h_im = h * im, hh_im = hh * im, h6_im = h6 * im;
  T cost = 0;
  for (int k0 = 0; k0 < N; k0 += 4) {
    // AHEAD: the controls of the group's four steps are read at its top
    // (indices clamped to the last step), so their loads wait once per group
    T uu[4][2];
    if constexpr (AHEAD) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kk = min(k0 + t, N - 1);
        uu[t][0] = ctrl(2 * kk);
        uu[t][1] = ctrl(2 * kk + 1);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + t;
      if (k >= N) break;  // uniform: every lane has the same horizon
      const T u0 = AHEAD ? uu[t][0] : ctrl(2 * k), u1 = AHEAD ? uu[t][1] : ctrl(2 * k + 1);
      if (!free_mass) {  // the end mass moves with the commanded velocity
        vx = u0;
        vy = u1;
      }
      T a_px, a_py, a_vx, a_vy, b_px, b_py, b_vx, b_vy;
      // a_v*, b_v*: tension differences (dv times the mass)
      chain_rhs<T, G>(px, py, vx, vy, cd, first, free_mass, a_px, a_py, a_vx, a_vy);
      T s_px = a_px, s_py = a_py, s_vx = a_vx, s_vy = a_vy;  // running k1 + 2 k2 + 2 k3 + k4
      chain_rhs<T, G>(px + hh * a_px, py + hh * a_py, vx + hh_im * a_vx, vy + hh_im * a_vy, cd,
                      first, free_mass, b_px, b_py, b_vx, b_vy);
      s_px += T(2) * b_px; s_py += T(2) * b_py; s_vx += T(2) * b_vx; s_vy += T(2) * b_vy;
      chain_rhs<T, G>(px + hh * b_px, py + hh * b_py, vx + hh_im * b_vx, vy + hh_im * b_vy, cd,
                      first, free_mass, a_px, a_py, a_vx, a_vy);
      s_px += T(2) * a_px; s_py += T(2) * a_py; s_vx += T(2) * a_vx; s_vy += T(2) * a_vy;
      chain_rhs<T, G>(px + h * a_px, py + h * a_py, vx + h_im * a_vx, vy + h_im * a_vy, cd, first,
                      free_mass, b_px, b_py, b_vx, b_vy);
      s_px += b_px; s_py += b_py; s_vx += b_vx; s_vy += b_vy;
      px += h6 * s_px;
      py += h6 * s_py;
      vx += h6_im * s_vx;
      vy += h6_im * s_vy;
      const T e0 = fma(wpx, px, cpx), e1 = fma(wpy, py, cpy);
      const T e2 = fma(wvx, vx, cvx), e3 = fma(wvy, vy, cvy);
      const T f0 = wu0 * u0, f1 = wu1 * u1;
      if constexpr (COST) {
        if (has_mass) cost += e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
        if (first) cost += f0 * f0 + f1 * f1;
      }
      sink.step(k, i, has_mass, first, e0, e1, e2, e3, f0, f1);
    }
  }
  if constexpr (COST) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) cost += __shfl_xor(cost, off, kWave);
  }
  return T(0.5) * cost;
}

// out[0] = (sum of v over the block of THREADS threads) / 2, in a fixed
// order; all threads of the block must call it.
template <typename T, int THREADS = kBlock>
__device__ __forceinline__ void block_half_sum(T v, T* out) {
  __shared__ T part[THREADS / kWave];
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
#pragma unroll
    for (int w = 0; w < THREADS / kWave; ++w) t += part[w];
    out[0] = T(0.5) * t;
  }
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Logical block g = (b % 8) * (gridDim.x / 8) + b / 8 gives each XCD
// a contiguous range of samples, so the neighbouring 64-byte row segments of
// adjacent blocks meet in the same L2 before they are written back.
__device__ __forceinline__ int xcd_logical_block() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Logical block g of one rollout launch: samples g kSpb .. g kSpb + kSpb - 1
// (column K is the nominal).  ctl_raw: the dynamic LDS for staged controls.
template <typename T, int G, int FL>
__device__ __forceinline__ void rollout_chain_block(
    ChainDev<T> cd, int N, const T* __restrict__ x0, const T* __restrict__ q,
    const T* __restrict__ r, const T* __restrict__ xref, const T* __restrict__ U,
    const T* __restrict__ W, int64_t ldw, int K, T* __restrict__ R, int64_t ldr,
    T* __restrict__ C, T* __restrict__ r0, T* __restrict__ c0, int nblocks, int stage_ctl, int g,
    unsigned char* ctl_raw) {
  constexpr int kSpb = kBlock / G;
  // residual staging tile of StagedSink (one allocation for both control paths)
  __shared__ T tile[2][FL * StagedSink<T, G, FL>::kRows][StagedSink<T, G, FL>::kLd];
  if (g >= nblocks) return;  // whole padding block: no barrier is shared with it
  const int ncol = K + (c0 ? 1 : 0);
  const int grp = threadIdx.x / G;
  const int gcol = g * kSpb + grp;
  const bool valid = gcol < ncol;
  const int col = valid ? gcol : ncol - 1;  // idle groups repeat a valid column, never store
  const bool nominal = col == K;
  const int n = 2 * N;
  // vector stores of residual rows need 4-element aligned rows
  const bool vec = R != nullptr && ldr % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(R) % (4 * sizeof(T)) == 0;
  const bool staged = R != nullptr || r0 != nullptr;
  const bool has_nominal = c0 != nullptr && g * kSpb <= K && K < (g + 1) * kSpb;  // uniform
  // cost terms in the rollout only where C is stored, or for a nominal whose
  // residual rows are not staged (with staged rows its c0 is the half sum of
  // squares that the sink collects)
  const bool want_cost = C != nullptr || (!staged && has_nominal);
  auto run = [&](const auto& ctrl, auto& sink) -> T {
    return want_cost ? chain_rollout<T, G, true>(cd, N, x0, q, r, xref, ctrl, sink)
                     : chain_rollout<T, G, false>(cd, N, x0, q, r, xref, ctrl, sink);
  };
  auto finish = [&](T c, T csum) {
    if (valid && (threadIdx.x & (G - 1)) == 0) {
      if (nominal) {
        if (!staged) c0[0] = c;
      } else if (C != nullptr) {
        C[col] = c;
      }
    }
    if (staged && has_nominal) block_half_sum(csum, c0);
  };
  auto go = [&](const auto& ctrl) {
    if (staged) {
      StagedSink<T, G, FL> sink{tile, R, ldr, r0, K, g * kSpb, cd.M, grp, N, vec};
      const T c = run(ctrl, sink);
      finish(c, sink.csum);
    } else {
      NoSink sink;
      finish(run(ctrl, sink), T(0));
    }
  };
  if (stage_ctl) {
    // the block's controls U + W[:, s] in one coalesced burst: ctl[idx][sample]
    T* ctl = reinterpret_cast<T*>(ctl_raw);
    const int col0 = g * kSpb;
    for (int e = threadIdx.x; e < n * kSpb; e += kBlock) {
      const int idx = e / kSpb, sl = e % kSpb;
      const int c = col0 + sl;
      T u = U[idx];
      if (W != nullptr && c < K) u += W[idx * ldw + c];
      ctl[e] = u;
    }
    __syncthreads();
    go(CtrlStaged<T>{ctl, kSpb, grp});
  } else {
    go(CtrlPerturbed<T>{U, W, ldw, (nominal || W == nullptr) ? -1 : col});
  }
}

template <typename T, int G>
__global__ void __launch_bounds__(256) rollout_chain_kernel(
    ChainDev<T> cd, int N, const T* __restrict__ x0, const T* __restrict__ q,
    const T* __restrict__ r, const T* __restrict__ xref, const T* __restrict__ U,
    const T* __restrict__ W, int64_t ldw, int K, T* __restrict__ R, int64_t ldr,
    T* __restrict__ C, T* __restrict__ r0, T* __restrict__ c0, int nblocks, int stage_ctl) {
  extern __shared__ unsigned char ctl_raw[];
  rollout_chain_block<T, G, staged_flush_steps<T, G>()>(cd, N, x0, q, r, xref, U, W, ldw, K, R,
                                                        ldr, C, r0, c0, nblocks, stage_ctl,
                                                        xcd_logical_block(), ctl_raw);
}

// Steps per flush of the split rollout: about 36 KB of LDS per buffer.
template <typename T, int G>
constexpr int split_flush_steps() {
  constexpr int per_step = (4 * G + 2) * (kBlock / G + 1) * static_cast<int>(sizeof(T));
  constexpr int f = 36864 / per_step;
  return f < 1 ? 1 : (f > 8 ? 8 : f);
}

// Single instance with residuals stored: 2 kBlock threads per block.  Waves
// 0-3 roll out the block's kSpb samples (as rollout_chain_kernel) and only
// fill the double-buffered residual tile in LDS; waves 4-7 drain each
// completed buffer to HBM while the rollout waves fill the other one.  At
// one rollout wave per SIMD a store that waits for the memory queue would
// hold up the RK4 steps of its SIMD; here it holds only a storing wave.
// Controls are staged in LDS (dynamic shared memory).
// Perturbations drawn by the rollout itself (Wout != nullptr): the draws of
// the sampler (gnmppi_sample with this key and stream, antithetic pairs when
// Kdraw < K), written to Wout for the later contraction while the block
// stages its controls U + W[:, s].
template <typename T>
struct RolloutDraw {
  T* Wout;
  T sigma;
  uint32_t k0, k1, s0, s1;
  int Kdraw;
};

template <typename T, int G, int F>
__global__ void __launch_bounds__(2 * kBlock) rollout_chain_split_kernel(
    ChainDev<T> cd, int N, const T* __restrict__ x0, const T* __restrict__ q,
    const T* __restrict__ r, const T* __restrict__ xref, const T* __restrict__ U,
    const T* __restrict__ W, int64_t ldw, int K, T* __restrict__ R, int64_t ldr,
    T* __restrict__ C, T* __restrict__ r0, T* __restrict__ c0, int nblocks,
    RolloutDraw<T> draw) {
  using Tile = ResidualTile<T, G, F>;
  constexpr int kSpb = Tile::kSpb;
  __shared__ T tile[2][F * Tile::kRows][Tile::kLd];
  extern __shared__ unsigned char ctl_raw[];
  const int g = xcd_logical_block();
  if (g >= nblocks) return;  // whole padding block: no barrier is shared with it
  const int col0 = g * kSpb;
  const int n = 2 * N;
  T* ctl = reinterpret_cast<T*>(ctl_raw);
  if (draw.Wout != nullptr) {
    // one Philox block (philox_rows<T>() rows) of one column per item
    constexpr int kr = philox_rows<T>();
    for (int e = threadIdx.x; e < (n + kr - 1) / kr * kSpb; e += 2 * kBlock) {
      const int b = e / kSpb, sl = e % kSpb, c = col0 + sl;
      const bool drawn = c < K;
      const bool mirror = c >= draw.Kdraw;  // antithetic partner of column c - Kdraw
      T v[kr];
      scaled_normals<T>(static_cast<uint32_t>(mirror ? c - draw.Kdraw : c),
                        static_cast<uint32_t>(b), draw.k0, draw.k1, draw.s0, draw.s1,
                        draw.sigma, v);
#pragma unroll
      for (int t = 0; t < kr; ++t) {
        const int row = kr * b + t;
        if (row < n) {
          const T w = mirror ? -v[t] : v[t];
          if (drawn) draw.Wout[row * ldw + c] = w;
          ctl[row * kSpb + sl] = drawn ? U[row] + w : U[row];
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < n * kSpb; e += 2 * kBlock) {
      const int idx = e / kSpb, sl = e % kSpb, c = col0 + sl;
      T u = U[idx];
      if (W != nullptr && c < K) u += W[idx * ldw + c];
      ctl[e] = u;
    }
  }
  __syncthreads();
  const bool has_nominal = c0 != nullptr && col0 <= K && K < col0 + kSpb;  // uniform
  T csum = 0;
  if (threadIdx.x < kBlock) {  // rollout waves (uniform per wave)
    const int grp = threadIdx.x / G;
    const int gcol = col0 + grp;
    TileSink<T, G, F> sink{tile, cd.M, grp, N};
    const CtrlStaged<T> ctrl{ctl, kSpb, grp};
    if (C != nullptr) {
      const T c = chain_rollout<T, G, true>(cd, N, x0, q, r, xref, ctrl, sink);
      if (gcol < K && (threadIdx.x & (G - 1)) == 0) C[gcol] = c;
    } else {
      chain_rollout<T, G, false>(cd, N, x0, q, r, xref, ctrl, sink);
    }
  } else {  // storing waves: one drain per barrier of the rollout waves
    const bool vec = R != nullptr && ldr % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(R) % (4 * sizeof(T)) == 0;
    const int rows = 4 * cd.M + 2;
    for (int k0 = 0; k0 < N; k0 += F) {
      __syncthreads();
      drain_tile<T, kSpb>(tile[(k0 / F) & 1], min(F, N - k0) * rows,
                          static_cast<int64_t>(k0) * rows, threadIdx.x - kBlock, R, ldr, r0, K,
                          col0, vec, csum);
    }
  }
  if (has_nominal) block_half_sum<T, 2 * kBlock>(csum, c0);
}

// Batched: item = (instance, logical block); controls always staged.  Fewer
// steps per flush than a single launch: several blocks share each CU.
constexpr int kBatchFlushSteps = 2;
template <int G>
__global__ void __launch_bounds__(256) batch_rollout_kernel(const BatchInst* __restrict__ inst,
                                                            BatchLaunch L, ChainDev<float> cd0) {
  extern __shared__ unsigned char ctl_raw[];
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    ChainDev<float> cd = cd0;
    cd.M = b.M;
    const int nblocks = ((b.K + 1) * G + kBlock - 1) / kBlock;
    rollout_chain_block<float, G, kBatchFlushSteps>(cd, b.N, b.x0, b.q, b.r, b.xref, b.U, b.W,
                                                    b.ldw, b.K, b.R, b.ldr, b.C, b.r0, b.c0,
                                                    nblocks, 1, it.tile, ctl_raw);
    __syncthreads();  // the next item reuses the LDS
  }
}

// Batched nominal rollout alone (the fused rollout-contraction path needs no
// nominal column): item = instance, the nominal U rolled out by one lane
// group; r0 and c0 as in the rollout above.
template <int G>
__global__ void __launch_bounds__(256) batch_nominal_kernel(const BatchInst* __restrict__ inst,
                                                            BatchLaunch L, ChainDev<float> cd0) {
  extern __shared__ unsigned char ctl_raw[];
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchInst& b = inst[L.items[w].inst];
    ChainDev<float> cd = cd0;
    cd.M = b.M;
    rollout_chain_block<float, G, kBatchFlushSteps>(cd, b.N, b.x0, b.q, b.r, b.xref, b.U, nullptr,
                                                    b.ldw, 0, nullptr, b.ldr, nullptr, b.r0, b.c0,
                                                    1, 1, 0, ctl_raw);
    __syncthreads();  // the next item reuses the LDS
  }
}

// ---- double integrator -----------------------------------------------------

template <typename T, int D, bool STORE, class Ctrl>
__device__ __forceinline__ T di_rollout(int N, T dt, const T* __restrict__ x0,
                                        const T* __restrict__ q, const T* __restrict__ r,
                                        const T* __restrict__ xref, const Ctrl& ctrl,
                                        T* __restrict__ R, int64_t ldr, int col, bool store_ok) {
  T p[D], v[D], wp[D], wv[D], wu[D], rp[D], rv[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    p[j] = x0[j];
    v[j] = x0[D + j];
    wp[j] = dsqrt(T(2) * q[j]);
    wv[j] = dsqrt(T(2) * q[D + j]);
    wu[j] = dsqrt(T(2) * r[j]);
    rp[j] = xref[j];
    rv[j] = xref[D + j];
  }
  const T hdt2 = T(0.5) * dt * dt;
  T cost = 0;
  if (N <= 0) return cost;
  // The raw control loads of a step are issued kAhead steps before it runs,
  // from indices clamped to the last step (unconditional, so no load sits in
  // a branch): the compiler cannot move a step's loads above the previous
  // step's residual stores, and without the ring every step would wait for
  // its own loads.  Whole turns of the ring run first; the last N % kAhead
  // steps then find their controls in the ring already.  The step's fused
  // multiply-adds are written out and no others are formed, so the storing
  // and the cost-only instantiations (the rollout's nominal and the line
  // search's chosen candidate) round alike.
  constexpr int kAhead = 8;
  auto step = [&](int k, const T (&u)[D]) {
#pragma clang fp contract(off)
    const int64_t base = static_cast<int64_t>(k) * 3 * D;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      p[j] = fma(hdt2, u[j], fma(dt, v[j], p[j]));
      v[j] = fma(dt, u[j], v[j]);
      const T e0 = wp[j] * (p[j] - rp[j]);
      const T e1 = wv[j] * (v[j] - rv[j]);
      const T e2 = wu[j] * u[j];
      cost += fma(e2, e2, fma(e1, e1, e0 * e0));
      if constexpr (STORE) {
        if (store_ok) {
          R[(base + j) * ldr + col] = e0;
          R[(base + D + j) * ldr + col] = e1;
          R[(base + 2 * D + j) * ldr + col] = e2;
        }
      }
    }
  };
  T la[kAhead][D], lb[kAhead][D];
#pragma unroll
  for (int s = 0; s < kAhead; ++s)
#pragma unroll
    for (int j = 0; j < D; ++j) ctrl.load(min(s, N - 1) * D + j, la[s][j], lb[s][j]);
  const int nfull = N - N % kAhead;
  for (int k0 = 0; k0 < nfull; k0 += kAhead) {
#pragma unroll
    for (int s = 0; s < kAhead; ++s) {
      const int kn = min(k0 + s + kAhead, N - 1);
      T u[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        u[j] = ctrl.value(la[s][j], lb[s][j]);
        ctrl.load(kn * D + j, la[s][j], lb[s][j]);
      }
      step(k0 + s, u);
    }
  }
  // ring slot s now holds step nfull + s
#pragma unroll
  for (int s = 0; s < kAhead; ++s) {
    if (nfull + s < N) {  // uniform
      T u[D];
#pragma unroll
      for (int j = 0; j < D; ++j) u[j] = ctrl.value(la[s][j], lb[s][j]);
      step(nfull + s, u);
    }
  }
  return T(0.5) * cost;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) rollout_di_kernel(
    int N, T dt, const T* __restrict__ x0, const T* __restrict__ q, const T* __restrict__ r,
    const T* __restrict__ xref, const T* __restrict__ U, const T* __restrict__ W, int64_t ldw,
    int K, T* __restrict__ R, int64_t ldr, T* __restrict__ C, T* __restrict__ r0,
    T* __restrict__ c0) {
  const int ncol = K + (c0 ? 1 : 0);
  const int col = blockIdx.x * kBlock + threadIdx.x;
  if (col >= ncol) return;  // no cross-lane traffic here, so idle lanes may leave
  const bool nominal = col == K;
  CtrlPerturbed<T> ctrl{U, W, ldw, (nominal || W == nullptr) ? -1 : col};
  T* out = nominal ? r0 : R;
  const int64_t ld = nominal ? 1 : ldr;
  const int ocol = nominal ? 0 : col;
  T c;
  if (out != nullptr)
    c = di_rollout<T, D, true>(N, dt, x0, q, r, xref, ctrl, out, ld, ocol, true);
  else
    c = di_rollout<T, D, false>(N, dt, x0, q, r, xref, ctrl, nullptr, 0, 0, false);
  if (nominal)
    c0[0] = c;
  else if (C != nullptr)
    C[col] = c;
}

// ---- line search (Eqs. (14)-(15)) -------------------------------------------

template <typename T>
__device__ __forceinline__ void line_select_and_apply(T* costs, int L, int n, T* U,
                                                      const T* __restrict__ dU,
                                                      const T* __restrict__ alpha,
                                                      T* __restrict__ Cout, double* info,
                                                      int32_t* status, int* jstar) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = -1;
    T bc = 0;
    for (int t = 0; t < L; ++t) {
      const T v = costs[t];
      if (finite(v) && (best < 0 || v < bc)) {
        best = t;
        bc = v;
      }
    }
    *jstar = best;
    if (Cout)
      for (int t = 0; t < L; ++t) Cout[t] = costs[t];
    if (info) {
      info[0] = best >= 0 ? static_cast<double>(alpha[best]) : 0.0;
      info[1] = best >= 0 ? static_cast<double>(bc) : __builtin_nan("");
      info[2] = static_cast<double>(best);
    }
    if (status) *status = best >= 0 ? GNMPPI_OK : GNMPPI_ENONFINITE;
  }
  __syncthreads();
  const int b = *jstar;
  if (b >= 0) {
    const T a = alpha[b];
    for (int t = threadIdx.x; t < n; t += blockDim.x) U[t] = U[t] + a * dU[t];
  }
}

// With Rc (the candidates' residual vectors, m apart): r0 <- the residuals of
// the chosen candidate and c0 <- its cost, i.e. the nominal residuals and cost
// of the updated controls (left as they are when no candidate is finite: U is
// unchanged then).  After line_select_and_apply, whose barrier orders the
// candidates' stores before these reads.
template <typename T>
__device__ __forceinline__ void line_nominal_out(const T* costs, int jstar, const T* Rc, int64_t m,
                                                 T* __restrict__ r0, T* __restrict__ c0) {
  if (Rc == nullptr || jstar < 0) return;  // uniform
  const T* src = Rc + jstar * m;
  // kBatch loads in flight per thread (clamped into the vector) before their
  // stores: one memory round trip per batch instead of one per element
  constexpr int kBatch = 16;
  const int64_t nt = blockDim.x;
  for (int64_t t0 = threadIdx.x; t0 < m; t0 += kBatch * nt) {
    T v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = src[min(t0 + u * nt, m - 1)];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (t0 + u * nt < m) r0[t0 + u * nt] = v[u];
  }
  if (threadIdx.x == 0) c0[0] = costs[jstar];
}

// With Rc, candidate j's residual rows go to Rc + j m and the chosen one's
// become r0 (line_nominal_out).
template <typename T, int G>
__device__ __forceinline__ void line_search_chain_block(
    ChainDev<T> cd, int N, const T* __restrict__ x0, const T* __restrict__ q,
    const T* __restrict__ r, const T* __restrict__ xref, T* U, const T* __restrict__ dU,
    const T* __restrict__ alpha, int L, T* __restrict__ Cout, double* info, int32_t* status,
    int stage_ctl, unsigned char* ctl_raw, T* __restrict__ Rc = nullptr,
    T* __restrict__ r0 = nullptr, T* __restrict__ c0 = nullptr) {
  __shared__ T costs[64];
  __shared__ int jstar;
  const int j = threadIdx.x / G;
  const int jj = j < L ? j : L - 1;
  const int n = 2 * N;
  const int64_t m = static_cast<int64_t>(N) * (4 * cd.M + 2);
  // groups past the last candidate repeat it and store nothing
  VectorSink<T> vsink{Rc != nullptr && j < L ? Rc + j * m : nullptr, cd.M};
  auto roll = [&](const auto& ctrl) {
    if (Rc != nullptr) return chain_rollout<T, G, true, true>(cd, N, x0, q, r, xref, ctrl, vsink);
    NoSink sink;
    return chain_rollout<T, G, true, true>(cd, N, x0, q, r, xref, ctrl, sink);
  };
  T c;
  if (stage_ctl) {
    T* Us = reinterpret_cast<T*>(ctl_raw);
    T* dUs = Us + n;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      Us[e] = U[e];
      dUs[e] = dU[e];
    }
    __syncthreads();
    c = roll(CtrlLineStaged<T>{Us, dUs, alpha[jj]});
  } else {
    c = roll(CtrlLine<T>{U, dU, alpha[jj]});
  }
  if (j < L && (threadIdx.x & (G - 1)) == 0) costs[j] = c;
  line_select_and_apply(costs, L, n, U, dU, alpha, Cout, info, status, &jstar);
  line_nominal_out(costs, jstar, Rc, m, r0, c0);
}

template <typename T, int G>
__global__ void __launch_bounds__(1024) line_search_chain_kernel(
    ChainDev<T> cd, int N, const T* __restrict__ x0, const T* __restrict__ q,
    const T* __restrict__ r, const T* __restrict__ xref, T* U, const T* __restrict__ dU,
    const T* __restrict__ alpha, int L, T* __restrict__ Cout, double* info, int32_t* status,
    int stage_ctl, T* __restrict__ Rc, T* __restrict__ r0, T* __restrict__ c0) {
  extern __shared__ unsigned char ctl_raw[];
  line_search_chain_block<T, G>(cd, N, x0, q, r, xref, U, dU, alpha, L, Cout, info, status,
                                stage_ctl, ctl_raw, Rc, r0, c0);
}

// Batched: item = instance; L * G threads.
template <int G>
__global__ void __launch_bounds__(1024) batch_line_search_kernel(const BatchInst* __restrict__ inst,
                                                                 BatchLaunch Lw, ChainDev<float> cd0,
                                                                 int L) {
  extern __shared__ unsigned char ctl_raw[];
  for (int w = blockIdx.x; w < Lw.count; w += gridDim.x) {
    const BatchInst& b = inst[Lw.items[w].inst];
    ChainDev<float> cd = cd0;
    cd.M = b.M;
    line_search_chain_block<float, G>(cd, b.N, b.x0, b.q, b.r, b.xref, b.U, b.dU, b.alpha, L,
                                      nullptr, b.info, b.status + 2, 1, ctl_raw);
    __syncthreads();
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(64) line_search_di_kernel(
    int N, T dt, const T* __restrict__ x0, const T* __restrict__ q, const T* __restrict__ r,
    const T* __restrict__ xref, T* U, const T* __restrict__ dU, const T* __restrict__ alpha,
    int L, T* __restrict__ Cout, double* info, int32_t* status, T* __restrict__ Rc,
    T* __restrict__ r0, T* __restrict__ c0) {
  __shared__ T costs[64];
  __shared__ int jstar;
  const int j = threadIdx.x;
  const int64_t m = static_cast<int64_t>(N) * 3 * D;
  if (j < L) {
    CtrlLine<T> ctrl{U, dU, alpha[j]};
    costs[j] = Rc != nullptr
                   ? di_rollout<T, D, true>(N, dt, x0, q, r, xref, ctrl, Rc + j * m, 1, 0, true)
                   : di_rollout<T, D, false>(N, dt, x0, q, r, xref, ctrl, nullptr, 0, 0, false);
  }
  line_select_and_apply(costs, L, N * D, U, dU, alpha, Cout, info, status, &jstar);
  line_nominal_out(costs, jstar, Rc, m, r0, c0);
}

// ---- dispatch ---------------------------------------------------------------

// Controls staged in LDS up to this size (the rest of the 160 KB holds the
// residual tile); larger horizons read them from global memory.
constexpr size_t kMaxStagedCtlBytes = 64 * 1024;

inline int chain_group(int M) {
  int g = 1;
  while (g < M) g <<= 1;
  return g;
}

template <typename T>
ChainDev<T> chain_dev(const gnmppi_problem& p) {
  return ChainDev<T>{p.n_masses, static_cast<T>(p.dt), static_cast<T>(p.k_lin),
                     static_cast<T>(p.k_cub), static_cast<T>(1.0 / p.mass)};
}

// With draw.Wout != nullptr (and W == nullptr) the perturbations are drawn
// in the same launch when the split kernel runs (staged controls, residuals
// wanted); otherwise the sampler runs first and the rollout reads its W.
template <typename T>
hipError_t rollout_typed(const gnmppi_problem& p, const T* x0, const T* U, const T* W,
                         int64_t ldw, int K, T* R, int64_t ldr, T* C, T* r0, T* c0,
                         hipStream_t st, RolloutDraw<T> draw = RolloutDraw<T>{}) {
  const T* q = static_cast<const T*>(p.q);
  const T* r = static_cast<const T*>(p.r);
  const T* xr = static_cast<const T*>(p.x_ref);
  const int ncol = K + (c0 ? 1 : 0);
  if (p.model == GNMPPI_MODEL_CHAIN) {
    const ChainDev<T> cd = chain_dev<T>(p);
    const int G = chain_group(p.n_masses);
    const int nblocks = (ncol * G + 255) / 256;
    dim3 grid((nblocks + 7) / 8 * 8);  // a multiple of the 8 XCDs, see xcd_logical_block()
    const size_t ctl_bytes = static_cast<size_t>(p.N) * 2 * (256 / G) * sizeof(T);
    const int stage = ctl_bytes <= kMaxStagedCtlBytes;
    const size_t lds = stage ? ctl_bytes : 0;
    // residuals with staged controls: the split kernel (rollout and storing
    // waves); costs only: the plain one
    const bool split = stage && (R != nullptr || r0 != nullptr);
    if (draw.Wout != nullptr && !split) {
      const uint64_t seed = (static_cast<uint64_t>(draw.k1) << 32) | draw.k0;
      const uint64_t sid = (static_cast<uint64_t>(draw.s1) << 32) | draw.s0;
      const hipError_t e = launch_sample(sizeof(T) == 4 ? GNMPPI_F32 : GNMPPI_F64, p.N * p.nu, K,
                                         static_cast<double>(draw.sigma), seed, sid,
                                         draw.Kdraw < K, draw.Wout, ldw, st);
      if (e != hipSuccess) return e;
      W = draw.Wout;
      draw.Wout = nullptr;
    }
#define GNM_CHAIN_CASE(GG)                                                                      \
  case GG:                                                                                      \
    if (split)                                                                                  \
      hipLaunchKernelGGL((rollout_chain_split_kernel<T, GG, split_flush_steps<T, GG>()>), grid, \
                         dim3(2 * kBlock), lds, st, cd, p.N, x0, q, r, xr, U, W, ldw, K, R, ldr, \
                         C, r0, c0, nblocks, draw);                                             \
    else                                                                                        \
      hipLaunchKernelGGL((rollout_chain_kernel<T, GG>), grid, dim3(kBlock), lds, st, cd, p.N,   \
                         x0, q, r, xr, U, W, ldw, K, R, ldr, C, r0, c0, nblocks, stage);        \
    break;
    switch (G) {
      GNM_CHAIN_CASE(1)
      GNM_CHAIN_CASE(2)
      GNM_CHAIN_CASE(4)
      GNM_CHAIN_CASE(8)
      GNM_CHAIN_CASE(16)
      default:
        return hipErrorInvalidValue;
    }
#undef GNM_CHAIN_CASE
  } else {
    dim3 grid((ncol + 255) / 256);
    const T dt = static_cast<T>(p.dt);
#define GNM_DI_CASE(DD)                                                                          \
  case DD:                                                                                       \
    hipLaunchKernelGGL((rollout_di_kernel<T, DD>), grid, dim3(256), 0, st, p.N, dt, x0, q, r, xr, \
                       U, W, ldw, K, R, ldr, C, r0, c0);                                         \
    break;
    switch (p.nu) {
      GNM_DI_CASE(1)
      GNM_DI_CASE(2)
      GNM_DI_CASE(3)
      GNM_DI_CASE(4)
      default:
        return hipErrorInvalidValue;
    }
#undef GNM_DI_CASE
  }
  return hipGetLastError();
}

template <typename T>
hipError_t line_search_typed(const gnmppi_problem& p, const T* x0, T* U, const T* dU,
                             const T* alpha, int L, T* C, double* info, int32_t* status,
                             hipStream_t st, T* Rc, T* r0, T* c0) {
  const T* q = static_cast<const T*>(p.q);
  const T* r = static_cast<const T*>(p.r);
  const T* xr = static_cast<const T*>(p.x_ref);
  if (p.model == GNMPPI_MODEL_CHAIN) {
    const ChainDev<T> cd = chain_dev<T>(p);
    const int G = chain_group(p.n_masses);
    const int threads = ((L * G + 63) / 64) * 64;
    const size_t ctl_bytes = static_cast<size_t>(p.N) * 2 * 2 * sizeof(T);
    const int stage = ctl_bytes <= kMaxStagedCtlBytes;
    const size_t lds = stage ? ctl_bytes : 0;
#define GNM_LS_CASE(GG)                                                                          \
  case GG:                                                                                       \
    hipLaunchKernelGGL((line_search_chain_kernel<T, GG>), dim3(1), dim3(threads), lds, st, cd,    \
                       p.N, x0, q, r, xr, U, dU, alpha, L, C, info, status, stage, Rc, r0, c0);  \
    break;
    switch (G) {
      GNM_LS_CASE(1)
      GNM_LS_CASE(2)
      GNM_LS_CASE(4)
      GNM_LS_CASE(8)
      GNM_LS_CASE(16)
      default:
        return hipErrorInvalidValue;
    }
#undef GNM_LS_CASE
  } else {
    const T dt = static_cast<T>(p.dt);
#define GNM_LSD_CASE(DD)                                                                      \
  case DD:                                                                                    \
    hipLaunchKernelGGL((line_search_di_kernel<T, DD>), dim3(1), dim3(64), 0, st, p.N, dt, x0, q, \
                       r, xr, U, dU, alpha, L, C, info, status, Rc, r0, c0);                  \
    break;
    switch (p.nu) {
      GNM_LSD_CASE(1)
      GNM_LSD_CASE(2)
      GNM_LSD_CASE(3)
      GNM_LSD_CASE(4)
      default:
        return hipErrorInvalidValue;
    }
#undef GNM_LSD_CASE
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rollout(const gnmppi_problem& p, const void* x0, const void* U, const void* W,
                          int64_t ldw, int K, void* R, int64_t ldr, void* C, void* r0, void* c0,
                          hipStream_t st) {
  if (p.dtype == GNMPPI_F32)
    return rollout_typed<float>(p, static_cast<const float*>(x0), static_cast<const float*>(U),
                                static_cast<const float*>(W), ldw, K, static_cast<float*>(R), ldr,
                                static_cast<float*>(C), static_cast<float*>(r0),
                                static_cast<float*>(c0), st);
  return rollout_typed<double>(p, static_cast<const double*>(x0), static_cast<const double*>(U),
                               static_cast<const double*>(W), ldw, K, static_cast<double*>(R),
                               ldr, static_cast<double*>(C), static_cast<double*>(r0),
                               static_cast<double*>(c0), st);
}

hipError_t launch_sample_rollout(const gnmppi_problem& p, const void* x0, const void* U,
                                 double sigma, uint64_t seed, uint64_t stream_id, int antithetic,
                                 void* W, int64_t ldw, int K, void* R, int64_t ldr, void* C,
                                 void* r0, void* c0, hipStream_t st) {
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const uint32_t s0 = static_cast<uint32_t>(stream_id), s1 = static_cast<uint32_t>(stream_id >> 32);
  const int Kdraw = antithetic ? K / 2 : K;
  if (p.model != GNMPPI_MODEL_CHAIN) {
    // the one-lane-per-sample kernel reads W: sampler, then rollout
    const hipError_t e = launch_sample(p.dtype, p.N * p.nu, K, sigma, seed, stream_id, antithetic,
                                       W, ldw, st);
    if (e != hipSuccess) return e;
    return launch_rollout(p, x0, U, W, ldw, K, R, ldr, C, r0, c0, st);
  }
  if (p.dtype == GNMPPI_F32)
    return rollout_typed<float>(p, static_cast<const float*>(x0), static_cast<const float*>(U),
                                nullptr, ldw, K, static_cast<float*>(R), ldr,
                                static_cast<float*>(C), static_cast<float*>(r0),
                                static_cast<float*>(c0), st,
                                RolloutDraw<float>{static_cast<float*>(W),
                                                   static_cast<float>(sigma), k0, k1, s0, s1,
                                                   Kdraw});
  return rollout_typed<double>(p, static_cast<const double*>(x0), static_cast<const double*>(U),
                               nullptr, ldw, K, static_cast<double*>(R), ldr,
                               static_cast<double*>(C), static_cast<double*>(r0),
                               static_cast<double*>(c0), st,
                               RolloutDraw<double>{static_cast<double*>(W), sigma, k0, k1, s0, s1,
                                                   Kdraw});
}

int batch_chain_group(int M) { return chain_group(M); }

int batch_rollout_tiles(int M, int K) {
  const int G = chain_group(M);
  return ((K + 1) * G + kBlock - 1) / kBlock;
}

size_t batch_rollout_lds(int G, int N) { return static_cast<size_t>(N) * 2 * (kBlock / G) * sizeof(float); }

hipError_t launch_batch_rollout(int G, const BatchInst* inst, const BatchLaunch& L,
                                const gnmppi_problem& shared, int N_max, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  const ChainDev<float> cd = chain_dev<float>(shared);
  const size_t lds = batch_rollout_lds(G, N_max);
  switch (G) {
    case 4:
      hipLaunchKernelGGL(batch_rollout_kernel<4>, dim3(L.blocks), dim3(kBlock), lds, st, inst, L, cd);
      break;
    case 8:
      hipLaunchKernelGGL(batch_rollout_kernel<8>, dim3(L.blocks), dim3(kBlock), lds, st, inst, L, cd);
      break;
    case 16:
      hipLaunchKernelGGL(batch_rollout_kernel<16>, dim3(L.blocks), dim3(kBlock), lds, st, inst, L, cd);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_nominal(int G, const BatchInst* inst, const BatchLaunch& L,
                                const gnmppi_problem& shared, int N_max, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  const ChainDev<float> cd = chain_dev<float>(shared);
  const size_t lds = batch_rollout_lds(G, N_max);
  switch (G) {
    case 4:
      hipLaunchKernelGGL(batch_nominal_kernel<4>, dim3(L.blocks), dim3(kBlock), lds, st, inst, L,
                         cd);
      break;
    case 8:
      hipLaunchKernelGGL(batch_nominal_kernel<8>, dim3(L.blocks), dim3(kBlock), lds, st, inst, L,
                         cd);
      break;
    case 16:
      hipLaunchKernelGGL(batch_nominal_kernel<16>, dim3(L.blocks), dim3(kBlock), lds, st, inst, L,
                         cd);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_line_search(int G, const BatchInst* inst, const BatchLaunch& Lw,
                                    const gnmppi_problem& shared, int L, int N_max,
                                    hipStream_t st) {
  if (Lw.count == 0) return hipSuccess;
  const ChainDev<float> cd = chain_dev<float>(shared);
  const int threads = ((L * G + 63) / 64) * 64;
  const size_t lds = static_cast<size_t>(N_max) * 2 * 2 * sizeof(float);
  switch (G) {
    case 4:
      hipLaunchKernelGGL(batch_line_search_kernel<4>, dim3(Lw.blocks), dim3(threads), lds, st, inst,
                         Lw, cd, L);
      break;
    case 8:
      hipLaunchKernelGGL(batch_line_search_kernel<8>, dim3(Lw.blocks), dim3(threads), lds, st, inst,
                         Lw, cd, L);
      break;
    case 16:
      hipLaunchKernelGGL(batch_line_search_kernel<16>, dim3(Lw.blocks), dim3(threads), lds, st,
                         inst, Lw, cd, L);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_line_search(const gnmppi_problem& p, const void* x0, void* U, const void* dU,
                              const void* alpha, int L, void* C, double* info, int32_t* status,
                              hipStream_t st, void* Rc, void* r0, void* c0) {
  if (p.dtype == GNMPPI_F32)
    return line_search_typed<float>(p, static_cast<const float*>(x0), static_cast<float*>(U),
                                    static_cast<const float*>(dU),
                                    static_cast<const float*>(alpha), L, static_cast<float*>(C),
                                    info, status, st, static_cast<float*>(Rc),
                                    static_cast<float*>(r0), static_cast<float*>(c0));
  return line_search_typed<double>(p, static_cast<const double*>(x0), static_cast<double*>(U),
                                   static_cast<const double*>(dU),
                                   static_cast<const double*>(alpha), L, static_cast<double*>(C),
                                   info, status, st, static_cast<double*>(Rc),
                                   static_cast<double*>(r0), static_cast<double*>(c0));
}

}  // namespace gnm
