// Dense n x n algebra of the Jacobian reconstruction (Eq. (10)) and of the
// GGN step (Eq. (13)), in double precision.
//
//  * reduce_sym_kernel -- adds the k-split / row-chunk partial sums of a
//      symmetric matrix (lower triangle) into a full symmetric double matrix,
//      one block per row so that every partial load is in flight at once.
//  * sweep_kernel<R> (sweep.hpp, instantiated in the sweep_*.hip units) --
//      one workgroup of 8 waves sweeps an SPD matrix with
//      the symmetric sweep operator (Gauss-Jordan elimination without
//      pivoting; for an SPD matrix its pivots are the Cholesky pivots
//      squared).  The lower triangle lives in registers as 16 x 16 tiles of
//      the f64 MFMA accumulator layout, whole tile rows per wave 1..7.
//      Pivots go in blocks of 16: wave 0 sweeps each diagonal block in
//      registers (two pivots per step), waves 1..7 apply the rank-16 update
//      of the previous block on the MFMA meanwhile -- one barrier per block.
//      Sweeping pivots 0..n-1 of [[H, g], [g^T, c]] leaves -H^{-1} in the
//      leading block and H^{-1} g in the last row: the same kernel yields
//      G^{-1} for the LS Jacobian and the GGN direction -(H^{-1} g) with no
//      triangular solves.  A pivot at or below n 2^-52 max diag marks the
//      matrix as not positive definite.
//  * reduce_rows_kernel / reduce_rows_vec_kernel -- S (or, for MC,
//      J = S / (K sigma^2)) as the sum of the k-split partials of the sample
//      contraction; J = S G^{-1}, where it is formed, runs on the MFMA
//      contraction kernel.
//  * gram_pair_kernel / batch_gram_kernel<NT> -- the lower tiles of
//      [A r0]^T [A r0] (A = J, or S for the direction without J) over a
//      chunk of rows with the 16x16x4 f64 MFMA (products of float inputs are
//      exact in double); one partial sum per chunk.
#include <mutex>
#include <type_traits>

#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace gnm {

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

using f64x4 = double __attribute__((ext_vector_type(4)));

// ---- partial-sum reduction -------------------------------------------------

// (G G)[i][j] for the symmetric n x n G (row-major), in a fixed order, so
// that entries (i, j) and (j, i) are bitwise equal.
__device__ __forceinline__ double gram_square_entry(const double* __restrict__ G, int n, int i,
                                                    int j) {
  const double* gi = G + static_cast<int64_t>(i) * n;
  double s0 = 0.0, s1 = 0.0;
  int k = 0;
  for (; k + 2 <= n; k += 2) {
    s0 = fma(gi[k], G[static_cast<int64_t>(k) * n + j], s0);
    s1 = fma(gi[k + 1], G[static_cast<int64_t>(k + 1) * n + j], s1);
  }
  if (k < n) s0 = fma(gi[k], G[static_cast<int64_t>(k) * n + j], s0);
  return s0 + s1;
}

// out (P x P, full, symmetric) = sum_sp part[sp] (rows row0.., leading dim ldp),
// reading only entries j <= i; diag_shift is added to the first npiv diagonal
// entries and, with Gsq != nullptr, lam_sq (Gsq Gsq)[i][j] (Gsq: npiv x npiv)
// to the leading npiv x npiv block.  grid.x = P (one row each), block = 256 >= P.
template <typename TP>
__device__ __forceinline__ void reduce_sym_row(const TP* __restrict__ part, int nsplit,
                                               int64_t split_stride, int row0, int ldp, int P,
                                               int npiv, double diag_shift,
                                               double* __restrict__ out, int i,
                                               const double* __restrict__ Gsq = nullptr,
                                               double lam_sq = 0.0) {
  const int j = threadIdx.x;
  if (j > i) return;
  const TP* src = part + static_cast<int64_t>(row0 + i) * ldp + j;
  // 16 independent loads per round (one L2 round trip per 16 partials), then
  // a fixed-order pairwise sum of the 16 accumulators
  constexpr int U = 16;
  double acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = 0.0;
  for (int sp = 0; sp < nsplit; sp += U) {
    TP v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = sp + u < nsplit ? src[(sp + u) * split_stride] : TP(0);
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] += static_cast<double>(v[u]);
  }
#pragma unroll
  for (int w = U / 2; w >= 1; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
  double s = acc[0];
  if (i == j && i < npiv) s += diag_shift;
  if (Gsq != nullptr && i < npiv) s += lam_sq * gram_square_entry(Gsq, npiv, i, j);
  out[static_cast<int64_t>(i) * P + j] = s;
  out[static_cast<int64_t>(j) * P + i] = s;
}

template <typename TP>
__global__ void __launch_bounds__(256) reduce_sym_kernel(const TP* __restrict__ part, int nsplit,
                                                         int64_t split_stride, int row0, int ldp,
                                                         int P, int npiv, double diag_shift,
                                                         double* __restrict__ out,
                                                         const double* __restrict__ Gsq,
                                                         double lam_sq) {
  reduce_sym_row<TP>(part, nsplit, split_stride, row0, ldp, P, npiv, diag_shift, out, blockIdx.x,
                     Gsq, lam_sq);
}

// Batched: MODE 0 reduces the G = W W^T partials into Gsum (P = n), MODE 1
// the [S r0]^T [S r0] partials into Hsum (P = n + 1, plus lambda G^2 in the
// leading n x n block).  tile = row i.
template <int MODE>
__global__ void __launch_bounds__(256) batch_reduce_sym_kernel(const BatchInst* __restrict__ inst,
                                                               BatchLaunch L, double lm_lambda) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    if constexpr (MODE == 0)
      reduce_sym_row<float>(b.gpart, b.gsplit, static_cast<int64_t>(b.n) * b.npad, 0, b.npad, b.n,
                            b.n, 0.0, b.Gsum, it.tile);
    else
      reduce_sym_row<double>(b.hpart, b.hsplit, static_cast<int64_t>(b.n + 1) * (b.n + 1), 0,
                             b.n + 1, b.n + 1, b.n, 0.0, b.Hsum, it.tile,
                             lm_lambda > 0.0 ? b.Gsum : nullptr, lm_lambda);
  }
}

// ---- S = sum of the k-split partials ------------------------------------------

// out[i, c] = scale * sum_sp part[sp][i, c] for i < m, c < n: 4 rows x 64
// columns per block, one element per thread, all partial loads in flight.
template <typename T>
__device__ __forceinline__ void reduce_rows_block(const T* __restrict__ part, int nsplit,
                                                  int64_t split_stride, int ldp, int m, int n,
                                                  double scale, T* __restrict__ out, int64_t ldo,
                                                  int32_t* status, int bx, int by) {
  if (status && bx == 0 && by == 0 && threadIdx.x == 0) *status = GNMPPI_OK;
  const int i = by * 4 + (threadIdx.x >> 6);
  const int c = bx * 64 + (threadIdx.x & 63);
  if (i >= m || c >= n) return;
  const T* src = part + static_cast<int64_t>(i) * ldp + c;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int sp = 0;
  for (; sp + 4 <= nsplit; sp += 4) {
    s0 += static_cast<double>(src[(sp + 0) * split_stride]);
    s1 += static_cast<double>(src[(sp + 1) * split_stride]);
    s2 += static_cast<double>(src[(sp + 2) * split_stride]);
    s3 += static_cast<double>(src[(sp + 3) * split_stride]);
  }
  for (; sp < nsplit; ++sp) s0 += static_cast<double>(src[sp * split_stride]);
  out[i * ldo + c] = static_cast<T>(((s0 + s1) + (s2 + s3)) * scale);
}

template <typename T>
__global__ void __launch_bounds__(256) reduce_rows_kernel(const T* __restrict__ part, int nsplit,
                                                          int64_t split_stride, int ldp, int m,
                                                          int n, double scale, T* __restrict__ out,
                                                          int64_t ldo, int32_t* status) {
  reduce_rows_block<T>(part, nsplit, split_stride, ldp, m, n, scale, out, ldo, status, blockIdx.x,
                       blockIdx.y);
}

// Sum of the k-slices (rows x npad each, slice stride rows * npad) over all
// npad columns, in slice order in double precision: rows i < m go to the FP32
// S (scaled by `scale`), rows m <= i < rows -- the rows of G = W W^T when the
// contraction carried them -- to the double ng x ng Gsum (columns < ng).
// tile = row group * ceil(npad / 64) + column group, 16 rows x 64 columns per
// block, four columns per thread with 16-byte loads, eight slices in flight.
__device__ __forceinline__ void reduce_rows_vec(const float* __restrict__ part, int nsplit,
                                                int rows, int m, int npad, double scale,
                                                float* __restrict__ S, int ng,
                                                double* __restrict__ Gsum, int tile) {
  using f32x4 = float __attribute__((ext_vector_type(4)));
  const int xb = (npad + 63) / 64;
  const int i = (tile / xb) * 16 + (threadIdx.x >> 4);
  const int c = (tile % xb) * 64 + 4 * (threadIdx.x & 15);
  if (i >= rows || c >= npad) return;
  const int64_t stride = static_cast<int64_t>(rows) * npad;
  const float* src = part + static_cast<int64_t>(i) * npad + c;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  constexpr int U = 8;
  for (int sp = 0; sp < nsplit; sp += U) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = sp + u < nsplit ? *reinterpret_cast<const f32x4*>(src + (sp + u) * stride)
                             : f32x4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a0 += static_cast<double>(v[u][0]);
      a1 += static_cast<double>(v[u][1]);
      a2 += static_cast<double>(v[u][2]);
      a3 += static_cast<double>(v[u][3]);
    }
  }
  if (i < m) {
    *reinterpret_cast<f32x4*>(S + static_cast<int64_t>(i) * npad + c) =
        f32x4{static_cast<float>(a0 * scale), static_cast<float>(a1 * scale),
              static_cast<float>(a2 * scale), static_cast<float>(a3 * scale)};
  } else {
    double* g = Gsum + static_cast<int64_t>(i - m) * ng + c;
    if (c + 0 < ng) g[0] = a0;
    if (c + 1 < ng) g[1] = a1;
    if (c + 2 < ng) g[2] = a2;
    if (c + 3 < ng) g[3] = a3;
  }
}

__global__ void __launch_bounds__(256) reduce_rows_vec_kernel(const float* __restrict__ part,
                                                              int nsplit, int rows, int m,
                                                              int npad, double scale,
                                                              float* __restrict__ S, int ng,
                                                              double* __restrict__ Gsum) {
  reduce_rows_vec(part, nsplit, rows, m, npad, scale, S, ng, Gsum, blockIdx.x);
}

// Batched: the slices of every instance (the padding columns of every slice
// are zero), with the rows of G below those of S where the fused rollout
// formed them.
__global__ void __launch_bounds__(256) batch_reduce_rows_kernel(const BatchInst* __restrict__ inst,
                                                                BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    reduce_rows_vec(b.part, b.nsplit, b.m + b.grows, b.m, b.npad, 1.0, b.S, b.n,
                    b.grows > 0 ? b.Gsum : nullptr, it.tile);
  }
}

// ---- [A r0]^T [A r0] with the f64 MFMA (A = J, or S) ------------------------------

// f64 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element j of lane l is D[4 j + l / 16][l % 16].
template <typename T, int NT>
__device__ __forceinline__ void gram_chunk(int m, int n, const T* __restrict__ J, int64_t ldj,
                                           const T* __restrict__ r0, int64_t inc, int chunk, int P,
                                           double* __restrict__ part, int bx) {
  constexpr int NPAIR = NT * (NT + 1) / 2;
  constexpr int NACC = (NPAIR + 3) / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ibeg = bx * chunk, iend = min(m, ibeg + chunk);
  f64x4 acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = f64x4{0, 0, 0, 0};
  // row k0 + kq of [J r0], columns 16 t + r16 (zero outside the chunk).
  // Branch-free: every lane loads from a clamped in-range address and the
  // value is selected afterwards, so the loads of one step are in flight
  // together instead of each waiting in its own branch.
  auto load = [&](int k0, T (&x)[NT]) {
    const int row = k0 + kq;
    const int64_t rr = min(row, m - 1);
    const T vr = r0[rr * inc];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = 16 * t + r16;
      const T vj = J[rr * ldj + min(col, n - 1)];
      const T v = col < n ? vj : (col == n ? vr : T(0));
      x[t] = row < iend ? v : T(0);
    }
  };
  // the next step's rows are requested before this step's MFMAs
  T cur[NT];
  load(ibeg, cur);
  for (int k0 = ibeg; k0 < iend; k0 += 4) {
    T nxt[NT];
    load(k0 + 4, nxt);
    double x[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) x[t] = static_cast<double>(cur[t]);
    int q = 0;
#pragma unroll
    for (int ta = 0; ta < NT; ++ta)
#pragma unroll
      for (int tb = 0; tb <= ta; ++tb, ++q)
        if ((q & 3) == wave)
          acc[q >> 2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[ta], x[tb], acc[q >> 2], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) cur[t] = nxt[t];
  }
  double* out = part + static_cast<int64_t>(bx) * P * P;
  int q = 0;
#pragma unroll
  for (int ta = 0; ta < NT; ++ta)
#pragma unroll
    for (int tb = 0; tb <= ta; ++tb, ++q)
      if ((q & 3) == wave) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 16 * ta + 4 * j + kq, b = 16 * tb + r16;
          if (a < P && b < P) out[static_cast<int64_t>(a) * P + b] = acc[q >> 2][j];
        }
      }
}

// Batched [S r0]^T [S r0] partials; tile = row chunk.
template <int NT>
__global__ void __launch_bounds__(256) batch_gram_kernel(const BatchInst* __restrict__ inst,
                                                         BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    gram_chunk<float, NT>(b.m, b.n, b.S, b.npad, b.r0, 1, b.hchunk, b.n + 1, b.hpart, it.tile);
  }
}

// Single instance: one block per (tile pair, row chunk).  Tile pair q is
// (ta, tb), tb <= ta, in the order (0,0), (1,0), (1,1), (2,0), ...; the four
// waves take interleaved 4-row steps of the chunk with all of their loads in
// flight at once (kGramSteps per wave), two accumulator chains per wave, and
// the wave sums are added in wave order.  One partial P x P matrix (lower
// tiles) per chunk.
constexpr int kGramSteps = 16;              // 4-row MFMA steps per wave and chunk
constexpr int kGramChunk = 16 * kGramSteps;  // rows per chunk (4 waves x 4 rows x steps)

template <typename T>
__global__ void __launch_bounds__(256) gram_pair_kernel(int m, int n, const T* __restrict__ J,
                                                        int64_t ldj, const T* __restrict__ r0,
                                                        int64_t inc, int P,
                                                        double* __restrict__ part) {
  __shared__ double red[4][256];
  int q = blockIdx.x, ta = 0;
  while (q > ta) {
    q -= ta + 1;
    ++ta;
  }
  const int tb = q;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ibeg = blockIdx.y * kGramChunk, iend = min(m, ibeg + kGramChunk);
  // Branch-free loads from clamped in-range addresses (the value is selected
  // afterwards), so all of a wave's loads are in flight together.
  const int ca = 16 * ta + r16, cb = 16 * tb + r16;
  T ja[kGramSteps], jb[kGramSteps], jr[kGramSteps];
#pragma unroll
  for (int u = 0; u < kGramSteps; ++u) {
    const int64_t rr = min(ibeg + 16 * u + 4 * wave + kq, m - 1);
    ja[u] = J[rr * ldj + min(ca, n - 1)];
    jb[u] = J[rr * ldj + min(cb, n - 1)];
    jr[u] = r0[rr * inc];
  }
  auto pick = [&](int u, int col, T vj) -> double {
    const int row = ibeg + 16 * u + 4 * wave + kq;
    const T v = col < n ? vj : (col == n ? jr[u] : T(0));
    return row < iend ? static_cast<double>(v) : 0.0;
  };
  f64x4 acc[2] = {f64x4{0, 0, 0, 0}, f64x4{0, 0, 0, 0}};
#pragma unroll
  for (int u = 0; u < kGramSteps; ++u)
    acc[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pick(u, ca, ja[u]), pick(u, cb, jb[u]),
                                                      acc[u & 1], 0, 0, 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) red[wave][64 * j + lane] = acc[0][j] + acc[1][j];
  __syncthreads();
  const int e = threadIdx.x, j = e >> 6, l = e & 63;
  const int a = 16 * ta + 4 * j + (l >> 4), b = 16 * tb + (l & 15);
  if (a < P && b < P) {
    const double v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    part[static_cast<int64_t>(blockIdx.y) * P * P + static_cast<int64_t>(a) * P + b] = v;
  }
}

template <typename T>
hipError_t launch_gram_pairs(int tiles, int nchunks, hipStream_t st, int m, int n, const T* J,
                             int64_t ldj, const T* r0, int64_t inc, int P, double* part) {
  const int pairs = tiles * (tiles + 1) / 2;
  hipLaunchKernelGGL(gram_pair_kernel<T>, dim3(pairs, nchunks), dim3(256), 0, st, m, n, J, ldj, r0,
                     inc, P, part);
  return hipGetLastError();
}

}  // namespace

// k-split of a contraction over `rows` output rows: every wave owns a 16-row
// tile and one of the kw step sequences of a slice; aim at ~4k waves (4 per
// SIMD) with at least two steps per wave and steps spread evenly.
static void split_plan(int rows, int K, int step, int kw, int& nsplit_out, int& split_len_out) {
  const int waves_per_split = (rows + 15) / 16 * kw;
  const int ksteps = (K + step - 1) / step;
  int nsplit = (4096 + waves_per_split - 1) / waves_per_split;
  const int max_split = ksteps / (2 * kw) > 1 ? ksteps / (2 * kw) : 1;
  if (nsplit > max_split) nsplit = max_split;
  if (nsplit < 1) nsplit = 1;
  int steps_per_split = (ksteps + nsplit - 1) / nsplit;
  steps_per_split = (steps_per_split + kw - 1) / kw * kw;
  nsplit_out = (ksteps + steps_per_split - 1) / steps_per_split;
  split_len_out = steps_per_split * step;
}

// k-split of the BF16 contraction: blocks of 64 bf16_row_tiles(terms) rows;
// aim at kBf16BlockTarget blocks (terms = 3) or kBf16BlockTargetPlain
// (terms = 1, a third of the MFMA work per step: fewer, longer blocks stream
// R better and write fewer partials) with at least four k-steps per block,
// and a whole number of turns of the kernel's load ring per slice.  The plain
// plan's 64-row k-slices are no more than the BF16x3 plan's, so terms = 3
// gives the larger split count.
static void bf16_split_plan(int m, int K, int terms, int& nsplit_out, int& split_len_out) {
  static_assert(kBf16BlockTargetPlain * kBf16RowTilesPlain <= kBf16BlockTarget * kBf16RowTiles,
                "workspace sized for terms = 3");
  const int rt = bf16_row_tiles(terms);
  const int row_blocks = (m + 64 * rt - 1) / (64 * rt);
  const int ksteps = (K + 31) / 32;
  const int target = terms == 3 ? kBf16BlockTarget : kBf16BlockTargetPlain;
  int nsplit = (target + row_blocks - 1) / row_blocks;
  const int max_split = ksteps / 4 > 1 ? ksteps / 4 : 1;
  if (nsplit > max_split) nsplit = max_split;
  if (nsplit < 1) nsplit = 1;
  int steps_per_split = (ksteps + nsplit - 1) / nsplit;
  steps_per_split = (steps_per_split + kBf16Depth - 1) / kBf16Depth * kBf16Depth;
  nsplit_out = (ksteps + steps_per_split - 1) / steps_per_split;
  split_len_out = steps_per_split * 32;
}

JacPlan jacobian_plan(int dtype, int m, int n, int K, int method) {
  JacPlan p{};
  const int esz = dtype == GNMPPI_F32 ? 4 : 8;
  const int step = dtype == GNMPPI_F32 ? 32 : 16;
  p.ncol_tiles = (n + 15) / 16;
  p.npad = 16 * p.ncol_tiles;
  const int base = method & 0xff;
  const bool ready = (method & GNMPPI_JAC_GRAM_READY) != 0;
  const int kw = contract_kw(esz, n);
  p.rows = m + ((base == GNMPPI_JAC_LS && !ready) ? n : 0);
  split_plan(p.rows, K, step, kw, p.nsplit, p.split_len);
  // the partial-sum area is sized for the largest split count over the row
  // sets of every method (m + n, m, and m on the BF16 kernel) so that all
  // methods share one workspace layout
  int ns_max, sl_max, ns_m, sl_m, ns_b = 0, sl_b;
  split_plan(m + n, K, step, kw, ns_max, sl_max);
  split_plan(m, K, step, kw, ns_m, sl_m);
  if (dtype == GNMPPI_F32) bf16_split_plan(m, K, 3, ns_b, sl_b);
  if (ns_m > ns_max) ns_max = ns_m;
  if (ns_b > ns_max) ns_max = ns_b;
  const size_t part_elems = static_cast<size_t>(ns_max) * (m + n) * p.npad;
  p.part_bytes = align_up(part_elems * esz);
  p.gsum_off = p.part_bytes;
  p.ginv_off = p.gsum_off + align_up(static_cast<size_t>(n) * n * 8);
  p.s_off = p.ginv_off + align_up(static_cast<size_t>(n) * p.npad * esz);
  split_plan(n, K, step, kw, p.gsplit, p.gsplit_len);
  p.gpart_off = p.s_off + align_up(static_cast<size_t>(m) * p.npad * esz);
  p.kpad = (K + 31) / 32 * 32;
  p.total = p.gpart_off + align_up(static_cast<size_t>(p.gsplit) * n * p.npad * esz);
  if (method & (GNMPPI_JAC_BF16 | GNMPPI_JAC_BF16X3)) {
    p.rows = m;  // G is formed by the FP32 W-only contraction
    bf16_split_plan(m, K, (method & GNMPPI_JAC_BF16X3) ? 3 : 1, p.nsplit, p.split_len);
  }
  return p;
}

// G = W W^T reduced to a full double matrix and inverted into Ginv (n x npad).
template <typename T>
hipError_t gram_inverse_typed(const JacPlan& pl, int n, int K, const T* W, int64_t ldw,
                              char* wk, const T* part, int nsplit, int64_t split_stride, int row0,
                              int32_t* status, hipStream_t st) {
  double* Gsum = reinterpret_cast<double*>(wk + pl.gsum_off);
  T* Ginv = reinterpret_cast<T*>(wk + pl.ginv_off);
  hipLaunchKernelGGL(reduce_sym_kernel<T>, dim3(n), dim3(256), 0, st, part, nsplit, split_stride,
                     row0, pl.npad, n, n, 0.0, Gsum, static_cast<const double*>(nullptr), 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  (void)K;
  (void)W;
  (void)ldw;
  return launch_sweep(n, n, kSweepInverse, Gsum, Ginv, pl.npad, nullptr, status, GNMPPI_ERANK,
                         st);
}

template <typename T>
hipError_t gram_typed(int m, int n, int K, const T* W, int64_t ldw, void* work, int32_t* status,
                      hipStream_t st) {
  const int dtype = sizeof(T) == 4 ? GNMPPI_F32 : GNMPPI_F64;
  const JacPlan pl = jacobian_plan(dtype, m, n, K, GNMPPI_JAC_LS);
  char* wk = static_cast<char*>(work);
  T* gpart = reinterpret_cast<T*>(wk + pl.gpart_off);
  const int64_t split_stride = static_cast<int64_t>(n) * pl.npad;
  ContractArgs<T> c{n, n, n, K, W, ldw, nullptr, nullptr, 0, W, ldw, pl.gsplit_len,
                    gpart, pl.npad, split_stride, pl.npad};
  hipError_t e = launch_contract(c, pl.gsplit, st);
  if (e != hipSuccess) return e;
  return gram_inverse_typed<T>(pl, n, K, W, ldw, wk, gpart, pl.gsplit, split_stride, 0, status, st);
}

template <typename T>
hipError_t jacobian_typed(int m, int n, int K, const T* R, int64_t ldr, const T* r0, const T* W,
                          int64_t ldw, int method, double sigma2, T* J, int64_t ldj, void* work,
                          int32_t* status, hipStream_t st) {
  const int dtype = sizeof(T) == 4 ? GNMPPI_F32 : GNMPPI_F64;
  const JacPlan pl = jacobian_plan(dtype, m, n, K, method);
  const int base = method & 0xff;
  const bool ready = (method & GNMPPI_JAC_GRAM_READY) != 0;
  const bool s_only = (method & GNMPPI_JAC_S_ONLY) != 0;
  const bool apply_only = (method & GNMPPI_JAC_APPLY_ONLY) != 0;
  const int bf16_terms = (method & GNMPPI_JAC_BF16X3) ? 3 : (method & GNMPPI_JAC_BF16) ? 1 : 0;
  char* wk = static_cast<char*>(work);
  T* part = reinterpret_cast<T*>(wk);
  const int64_t split_stride = static_cast<int64_t>(pl.rows) * pl.npad;
  hipError_t e;
  if (!apply_only) {
    if constexpr (sizeof(T) == 4) {
      if (bf16_terms) {
        // S on the BF16 MFMA (W split on the fly); G (LS) on the FP32 W-only
        // contraction
        e = launch_contract_bf16(bf16_terms, m, n, K, R, ldr, r0, W, ldw, pl.nsplit, pl.split_len,
                                 part, pl.npad, st);
        if (e != hipSuccess) return e;
        if (base == GNMPPI_JAC_LS && !ready) {
          e = gram_typed<T>(m, n, K, W, ldw, work, status, st);
          if (e != hipSuccess) return e;
        }
      }
    }
    if (!bf16_terms) {
      // S = (R - r0 1^T) W^T and (LS, unless ready) G = W W^T, as k-split partial sums
      ContractArgs<T> c1{m, pl.rows, n, K, R, ldr, r0, W, ldw, W, ldw, pl.split_len,
                         part, pl.npad, split_stride, pl.npad};
      e = launch_contract(c1, pl.nsplit, st);
      if (e != hipSuccess) return e;
    }
    if (s_only) return hipSuccess;
    if (base == GNMPPI_JAC_MC) {
      const dim3 rgrid((n + 63) / 64, (m + 3) / 4);
      // MC has no factorisation that can fail: the reduction reports success
      hipLaunchKernelGGL(reduce_rows_kernel<T>, rgrid, dim3(256), 0, st, part, pl.nsplit,
                         split_stride, pl.npad, m, n, 1.0 / (static_cast<double>(K) * sigma2), J,
                         ldj, status);
      return hipGetLastError();
    }
    if (!ready && !bf16_terms) {
      e = gram_inverse_typed<T>(pl, n, K, W, ldw, wk, part, pl.nsplit, split_stride, m, status, st);
      if (e != hipSuccess) return e;
    }
  }
  // J = S G^{-1} = S (G^{-1})^T: the same contraction over the decision index,
  // with S = the sum of the k-slice partials added while the A operand loads.
  // With a ready G the rank check belongs to gnmppi_perturbation_gram's own
  // status word and this contraction reports success.
  T* Ginv = reinterpret_cast<T*>(wk + pl.ginv_off);
  ContractArgs<T> c2{m, m, n, n, part, pl.npad, nullptr, nullptr, 0, Ginv, pl.npad, n,
                     J, ldj, 0, n};
  c2.asplit = pl.nsplit;
  c2.asplit_stride = split_stride;
  c2.status = ready ? status : nullptr;
  return launch_contract(c2, 1, st);
}

hipError_t launch_gram(int dtype, int m, int n, int K, const void* W, int64_t ldw, void* work,
                       int32_t* status, hipStream_t st) {
  if (dtype == GNMPPI_F32)
    return gram_typed<float>(m, n, K, static_cast<const float*>(W), ldw, work, status, st);
  return gram_typed<double>(m, n, K, static_cast<const double*>(W), ldw, work, status, st);
}

hipError_t launch_jacobian(int dtype, int m, int n, int K, const void* R, int64_t ldr,
                           const void* r0, const void* W, int64_t ldw, int method, double sigma2,
                           void* J, int64_t ldj, void* work, int32_t* status, hipStream_t st) {
  if (dtype == GNMPPI_F32)
    return jacobian_typed<float>(m, n, K, static_cast<const float*>(R), ldr,
                                 static_cast<const float*>(r0), static_cast<const float*>(W), ldw,
                                 method, sigma2, static_cast<float*>(J), ldj, work, status, st);
  return jacobian_typed<double>(m, n, K, static_cast<const double*>(R), ldr,
                                static_cast<const double*>(r0), static_cast<const double*>(W), ldw,
                                method, sigma2, static_cast<double*>(J), ldj, work, status, st);
}

GgnPlan ggn_plan(int dtype, int m, int n) {
  (void)dtype;
  GgnPlan g{};
  g.P = n + 1;
  g.tiles = (g.P + 15) / 16;
  g.chunk = kGramChunk;
  g.nsplit = (m + kGramChunk - 1) / kGramChunk;
  g.part_bytes = align_up(static_cast<size_t>(g.nsplit) * g.P * g.P * 8);
  g.total = g.part_bytes + align_up(static_cast<size_t>(g.P) * g.P * 8);
  return g;
}

hipError_t launch_ggn(int dtype, int m, int n, const void* J, int64_t ldj, const void* r0,
                      int64_t inc_r0, double lm_lambda, void* dU, void* work, int32_t* status,
                      hipStream_t st) {
  const GgnPlan g = ggn_plan(dtype, m, n);
  double* part = static_cast<double*>(work);
  double* Hsum = reinterpret_cast<double*>(static_cast<char*>(work) + g.part_bytes);
  hipError_t e;
  if (dtype == GNMPPI_F32)
    e = launch_gram_pairs<float>(g.tiles, g.nsplit, st, m, n, static_cast<const float*>(J), ldj,
                                 static_cast<const float*>(r0), inc_r0, g.P, part);
  else
    e = launch_gram_pairs<double>(g.tiles, g.nsplit, st, m, n, static_cast<const double*>(J), ldj,
                                  static_cast<const double*>(r0), inc_r0, g.P, part);
  if (e != hipSuccess) return e;
  const int64_t split_stride = static_cast<int64_t>(g.P) * g.P;
  hipLaunchKernelGGL(reduce_sym_kernel<double>, dim3(g.P), dim3(256), 0, st, part, g.nsplit,
                     split_stride, 0, g.P, g.P, n, lm_lambda, Hsum,
                     static_cast<const double*>(nullptr), 0.0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == GNMPPI_F32)
    return launch_sweep(g.P, n, kSweepDirection, Hsum, nullptr, 0, static_cast<float*>(dU),
                               status, GNMPPI_ENOTPD, st);
  return launch_sweep(g.P, n, kSweepDirection, Hsum, nullptr, 0, static_cast<double*>(dU),
                              status, GNMPPI_ENOTPD, st);
}

// ---- the GGN direction without forming J ------------------------------------

// With J = S A (LS: A = G^{-1}; MC: A = I / (K sigma2)) and B = A^{-1},
// J^T J + lambda I = A (S^T S + lambda B^2) A and J^T r0 = A S^T r0, so the
// GGN direction is dU = B y with (S^T S + lambda B^2) y = -S^T r0.  LS runs
// that system: the normal matrix of [S r0] (plus lambda G^2), the sweep, and
// B = G applied to y inside the sweep, so J = S G^{-1} (an m x n x n
// contraction) is never formed.  Without a ready G the sample contraction
// carries the n rows of W as extra rows of its A operand, so G comes out of
// the same launch and the same slice reduction as S.  MC forms
// J = S / (K sigma2) in the slice reduction, then the plain GGN step.
// Workspace: the Jacobian workspace followed by the GGN workspace.
size_t ggn_direction_bytes(int dtype, int m, int n, int K) {
  return jacobian_plan(dtype, m, n, K, GNMPPI_JAC_LS).total + ggn_plan(dtype, m, n).total;
}

template <typename T>
hipError_t ggn_direction_typed(int m, int n, int K, const T* R, int64_t ldr, const T* r0,
                               const T* W, int64_t ldw, int method, double sigma2,
                               double lm_lambda, T* dU, void* work, int32_t* status,
                               hipStream_t st) {
  const int dtype = sizeof(T) == 4 ? GNMPPI_F32 : GNMPPI_F64;
  // the offsets of the regions (partials, G, S) and the workspace size
  const JacPlan pl = jacobian_plan(dtype, m, n, K, GNMPPI_JAC_LS);
  const int base = method & 0xff;
  const bool ls = base == GNMPPI_JAC_LS;
  const bool with_gram = ls && (method & GNMPPI_JAC_GRAM_READY) == 0;
  const bool s_only = (method & GNMPPI_JAC_S_ONLY) != 0;
  const bool apply_only = (method & GNMPPI_JAC_APPLY_ONLY) != 0;
  const int bf16_terms = (method & GNMPPI_JAC_BF16X3) ? 3 : (method & GNMPPI_JAC_BF16) ? 1 : 0;
  // rows of each k-slice: S, then (with_gram) G; the partial-sum region
  // holds the largest split count of every row set, so these fit
  const int rows = with_gram ? m + n : m;
  int nsplit = 0, split_len = 0;
  if (bf16_terms)
    bf16_split_plan(rows, K, bf16_terms, nsplit, split_len);
  else
    split_plan(rows, K, sizeof(T) == 4 ? 32 : 16, contract_kw(sizeof(T), n), nsplit, split_len);
  char* wk = static_cast<char*>(work);
  T* part = reinterpret_cast<T*>(wk);
  const int64_t split_stride = static_cast<int64_t>(rows) * pl.npad;
  double* Gsum = reinterpret_cast<double*>(wk + pl.gsum_off);
  hipError_t e = hipSuccess;
  if (!apply_only) {
    if constexpr (sizeof(T) == 4) {
      if (bf16_terms)
        e = launch_contract_bf16(bf16_terms, m, n, K, R, ldr, r0, W, ldw, nsplit, split_len, part,
                                 pl.npad, st, with_gram);
    }
    if (!bf16_terms) {
      // A = [R - r0 1^T; W] (the W rows only with_gram), B = W
      ContractArgs<T> c1{m, rows, n, K, R, ldr, r0, W, ldw, W, ldw, split_len,
                         part, pl.npad, split_stride, pl.npad};
      e = launch_contract(c1, nsplit, st);
    }
    if (e != hipSuccess || s_only) return e;
  }
  // S (LS) or J (MC) from the slices, and G (with_gram)
  T* S = reinterpret_cast<T*>(wk + pl.s_off);
  const double scale = ls ? 1.0 : 1.0 / (static_cast<double>(K) * sigma2);
  if constexpr (sizeof(T) == 4) {
    hipLaunchKernelGGL(reduce_rows_vec_kernel, dim3(((rows + 15) / 16) * ((pl.npad + 63) / 64)),
                       dim3(256), 0, st, part, nsplit, rows, m, pl.npad, scale, S, n, Gsum);
  } else {
    const dim3 rgrid((n + 63) / 64, (m + 3) / 4);
    hipLaunchKernelGGL(reduce_rows_kernel<T>, rgrid, dim3(256), 0, st, part, nsplit,
                       split_stride, pl.npad, m, n, scale, S, static_cast<int64_t>(pl.npad),
                       static_cast<int32_t*>(nullptr));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (with_gram)
      hipLaunchKernelGGL(reduce_sym_kernel<T>, dim3(n), dim3(256), 0, st, part, nsplit,
                         split_stride, m, pl.npad, n, n, 0.0, Gsum,
                         static_cast<const double*>(nullptr), 0.0);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // normal matrix of [S r0] (of [J r0] for MC, lambda on its diagonal)
  const GgnPlan g = ggn_plan(dtype, m, n);
  char* gw = wk + pl.total;
  double* gpart = reinterpret_cast<double*>(gw);
  double* Hsum = reinterpret_cast<double*>(gw + g.part_bytes);
  e = launch_gram_pairs<T>(g.tiles, g.nsplit, st, m, n, S, pl.npad, r0, 1, g.P, gpart);
  if (e != hipSuccess) return e;
  // LS: + lambda G^2 (B = G); MC: + lambda on the diagonal
  hipLaunchKernelGGL(reduce_sym_kernel<double>, dim3(g.P), dim3(256), 0, st, gpart, g.nsplit,
                     static_cast<int64_t>(g.P) * g.P, 0, g.P, g.P, n, ls ? 0.0 : lm_lambda, Hsum,
                     ls && lm_lambda > 0.0 ? static_cast<const double*>(Gsum) : nullptr,
                     lm_lambda);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sweep(g.P, n, kSweepDirection, Hsum, nullptr, 0, dU, status, GNMPPI_ENOTPD, st,
                      ls ? static_cast<const double*>(Gsum) : nullptr, static_cast<int64_t>(n));
}

hipError_t launch_ggn_direction(int dtype, int m, int n, int K, const void* R, int64_t ldr,
                                const void* r0, const void* W, int64_t ldw, int method,
                                double sigma2, double lm_lambda, void* dU, void* work,
                                int32_t* status, hipStream_t st) {
  if (dtype == GNMPPI_F32)
    return ggn_direction_typed<float>(m, n, K, static_cast<const float*>(R), ldr,
                                      static_cast<const float*>(r0), static_cast<const float*>(W),
                                      ldw, method, sigma2, lm_lambda, static_cast<float*>(dU),
                                      work, status, st);
  return ggn_direction_typed<double>(m, n, K, static_cast<const double*>(R), ldr,
                                     static_cast<const double*>(r0), static_cast<const double*>(W),
                                     ldw, method, sigma2, lm_lambda, static_cast<double*>(dU),
                                     work, status, st);
}

// ---- the GGN step without a caller workspace ----------------------------------

// Scratch of gnmppi_ggn_step_noalloc: the [J r0]^T [J r0] chunk partials and
// the reduced normal matrix, in a file-scope device array (each GPU holds its
// own copy for the life of the process).  In host code `scratch` names a
// host-side stand-in, never the device memory: its device address comes from
// hipGetSymbolAddress, looked up once per device and kept in kScratchPtr.
constexpr size_t kNoAllocScratchBytes = size_t{8} << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex kScratchMutex;
void* kScratchPtr[kMaxDevices] = {};
}  // namespace

size_t ggn_noalloc_capacity() { return kNoAllocScratchBytes; }

// The current device's address of `scratch` (looked up on the first call on
// that device, with it current).
static hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(kScratchMutex);
  if (kScratchPtr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) return hipErrorInvalidSymbol;
    kScratchPtr[dev] = p;
  }
  *out = kScratchPtr[dev];
  return hipSuccess;
}

hipError_t launch_ggn_noalloc(int dtype, int m, int n, const void* J, int64_t ldj, const void* r0,
                              int64_t inc_r0, double lm_lambda, void* dU, int32_t* status,
                              hipStream_t st) {
  if (ggn_plan(dtype, m, n).total > kNoAllocScratchBytes) return hipErrorInvalidValue;
  void* work = nullptr;
  const hipError_t e = scratch_address(&work);
  if (e != hipSuccess) return e;
  // every element the step reads from its workspace is written earlier in
  // the same step (all chunk partials, both triangles of the normal
  // matrix), so nothing needs clearing between calls
  return launch_ggn(dtype, m, n, J, ldj, r0, inc_r0, lm_lambda, dU, work, status, st);
}

// ---- batched launchers ------------------------------------------------------

hipError_t launch_batch_reduce_sym(int mode, const BatchInst* inst, const BatchLaunch& L,
                                   double lm_lambda, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL(batch_reduce_sym_kernel<0>, dim3(L.blocks), dim3(256), 0, st, inst, L,
                       lm_lambda);
  else
    hipLaunchKernelGGL(batch_reduce_sym_kernel<1>, dim3(L.blocks), dim3(256), 0, st, inst, L,
                       lm_lambda);
  return hipGetLastError();
}

hipError_t launch_batch_sweep(int mode, int R, const BatchInst* inst, const BatchLaunch& L,
                              hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  return mode == 0 ? launch_batch_sweep_mode0(R, inst, L, st)
                   : launch_batch_sweep_mode1(R, inst, L, st);
}

hipError_t launch_batch_reduce_rows(const BatchInst* inst, const BatchLaunch& L, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_reduce_rows_kernel, dim3(L.blocks), dim3(256), 0, st, inst, L);
  return hipGetLastError();
}

hipError_t launch_batch_gram(int nt, const BatchInst* inst, const BatchLaunch& L, hipStream_t st) {
  if (L.count == 0) return hipSuccess;
#define GNM_BG_CASE(NT)                                                                          \
  case NT:                                                                                       \
    hipLaunchKernelGGL((batch_gram_kernel<NT>), dim3(L.blocks), dim3(256), 0, st, inst, L);       \
    break;
  switch (nt) {
    GNM_BG_CASE(1) GNM_BG_CASE(2) GNM_BG_CASE(3) GNM_BG_CASE(4) GNM_BG_CASE(5) GNM_BG_CASE(6)
    GNM_BG_CASE(7) GNM_BG_CASE(8) GNM_BG_CASE(9) GNM_BG_CASE(10) GNM_BG_CASE(11)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_BG_CASE
  return hipGetLastError();
}

}  // namespace gnm
