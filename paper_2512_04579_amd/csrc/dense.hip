// Dense n x n algebra of the Jacobian reconstruction (Eq. (10)) and of the
// GGN step (Eq. (13)), in double precision.
//
//  * reduce_sym_kernel -- adds the k-split / row-chunk partial sums of a
//      symmetric matrix (lower triangle) into a full symmetric double matrix,
//      one block per row so that every partial load is in flight at once.
//  * sweep_kernel<R> -- one workgroup of 4 waves sweeps an SPD matrix with
//      the symmetric sweep operator (Gauss-Jordan elimination without
//      pivoting; for an SPD matrix its pivots are the Cholesky pivots
//      squared).  The lower triangle lives in registers as 16 x 16 tiles of
//      the f64 MFMA accumulator layout, whole tile rows per wave 1..3.
//      Pivots go in blocks of 16: wave 0 sweeps each diagonal block in
//      registers (two pivots per step), waves 1..3 apply the rank-16 update
//      of the previous block on the MFMA meanwhile -- one barrier per block.
//      Sweeping pivots 0..n-1 of [[H, g], [g^T, c]] leaves -H^{-1} in the
//      leading block and H^{-1} g in the last row: the same kernel yields
//      G^{-1} for the LS Jacobian and the GGN direction -(H^{-1} g) with no
//      triangular solves.  A pivot at or below n 2^-52 max diag marks the
//      matrix as not positive definite.
//  * reduce_rows_kernel -- S (or, for MC, J = S / (K sigma^2)) as the sum of
//      the k-split partials of the sample contraction; J = S G^{-1} then runs
//      on the MFMA contraction kernel.
//  * gram_pair_kernel / batch_gram_kernel<NT> -- the lower tiles of
//      [J r0]^T [J r0] over a chunk of rows with the 16x16x4 f64 MFMA
//      (products of float inputs are exact in double); one partial sum per
//      chunk.
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

// out (P x P, full, symmetric) = sum_sp part[sp] (rows row0.., leading dim ldp),
// reading only entries j <= i; diag_shift is added to the first npiv diagonal
// entries.  grid.x = P (one row each), block = 256 >= P.
template <typename TP>
__device__ __forceinline__ void reduce_sym_row(const TP* __restrict__ part, int nsplit,
                                               int64_t split_stride, int row0, int ldp, int P,
                                               int npiv, double diag_shift,
                                               double* __restrict__ out, int i) {
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
  out[static_cast<int64_t>(i) * P + j] = s;
  out[static_cast<int64_t>(j) * P + i] = s;
}

template <typename TP>
__global__ void __launch_bounds__(256) reduce_sym_kernel(const TP* __restrict__ part, int nsplit,
                                                         int64_t split_stride, int row0, int ldp,
                                                         int P, int npiv, double diag_shift,
                                                         double* __restrict__ out) {
  reduce_sym_row<TP>(part, nsplit, split_stride, row0, ldp, P, npiv, diag_shift, out, blockIdx.x);
}

// Batched: MODE 0 reduces the G = W W^T partials into Gsum (P = n), MODE 1
// the [J r0]^T [J r0] partials into Hsum (P = n + 1, lambda on the first n
// diagonal entries).  tile = row i.
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
                             b.n + 1, b.n + 1, b.n, lm_lambda, b.Hsum, it.tile);
  }
}

// ---- blocked register-resident symmetric sweep ------------------------------

enum SweepOut { kSweepInverse = 0, kSweepDirection = 1 };

constexpr int kSweepTD = 16;  // thread grid edge = pivots per block
constexpr int kSweepLd = 18;  // LDS row stride (doubles): 16-byte rows, no bank conflicts

// Reciprocal of an FP64 pivot: the hardware estimate refined by two
// Newton-Raphson steps x <- x + x (1 - d x) (quadratic convergence; the
// result is within an ulp of 1/d).
__device__ __forceinline__ double recip(double d) {
  double x = __builtin_amdgcn_rcp(d);
  x = fma(fma(-d, x, 1.0), x, x);
  x = fma(fma(-d, x, 1.0), x, x);
  return x;
}

// Cross-lane moves of an FP64 value: a 64-bit DPP row_newbcast (every lane
// reads lane N of its 16-lane row), a broadcast of 16-lane row G to all four
// rows (every lane l reads lane l % 16 + 16 G) with the two lane-swap
// instructions, and a read of one lane into a uniform value.
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  // the builtin takes the type of its operands (one v_mov_b64_dpp here)
  long long b = __builtin_bit_cast(long long, v);
  const long long r = __builtin_amdgcn_update_dpp(b, b, 0x150 + N, 0xf, 0xf, false);
  return __builtin_bit_cast(double, r);
}
template <int G>
__device__ __forceinline__ int rows_bcast32(int v) {
  // swap32(v, v) = {rows 0 1 0 1, rows 2 3 2 3}; swap16(a, a) = {a0 a0 a2 a2, a1 a1 a3 a3}
  const auto h = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  const int a = G < 2 ? h[0] : h[1];
  const auto r = __builtin_amdgcn_permlane16_swap(a, a, false, false);
  return (G & 1) ? r[1] : r[0];
}
template <int G>
__device__ __forceinline__ double rows_bcast(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = rows_bcast32<G>(static_cast<int>(b));
  const int hi = rows_bcast32<G>(static_cast<int>(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// The sweep over one pivot p is the rank-1 update A <- A_{\p} - z z^T / d
// with d = A_pp, z = column p with its pivot entry replaced by -1, and
// A_{\p} = A with row and column p zeroed.  For a block B of pivots the same
// identity reads A <- A_{\B} - Z D^{-1} Z^T with D = A_BB and Z = A_{:,B}
// whose rows in B are replaced by -I; sweeping B inside D alone gives
// -D^{-1}.  diag_pivot<p> does one pivot of that on one wave: lane l holds
// D[l % 16][4 e + l / 16], e < 4 (the f64 MFMA accumulator layout of a
// symmetric tile), so row p of the block is lane p of every 16-lane row (a
// DPP broadcast), the pivot one lane (a readlane) and column p register
// p / 4 of 16-lane row p % 4 (a row broadcast).  Branch-free: pivots
// p >= nbv leave D as it is and a pivot at or below tol clears `ok`.
template <int p>
__device__ __forceinline__ void diag_pivot(double (&d4)[4], int nbv, double tol, bool& ok, int li,
                                           int lg) {
  constexpr int gp = p & 3, ep = p >> 2;
  const bool act = p < nbv;  // uniform
  const double d = read_lane(d4[ep], p + 16 * gp);
  ok = ok && (!act || d > tol);
  const double inv = recip(d);
  double zi = rows_bcast<gp>(d4[ep]);  // D[li][p]
  double zj[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) zj[e] = row_bcast<p>(d4[e]);  // D[p][4 e + lg]
  if (li == p) zi = -1.0;
  const double sr = act ? -zi * inv : 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool pc = 4 * e + lg == p;
    const double a = (act && (li == p || pc)) ? 0.0 : d4[e];
    d4[e] = fma(sr, pc ? -1.0 : zj[e], a);
  }
}

// Pivots p and p + 1 together: with the 2 x 2 block B = [[a, b], [b, c]] of
// D on them, D <- D_{\B} - Y Z^T where Z = columns p, p + 1 with rows p,
// p + 1 replaced by -I and Y = Z B^{-1}, B^{-1} = [[c, -b], [-b, a]] / det.
// One reciprocal per two pivots halves the latency chain of the single
// pivots (the same block identity as between diagonal blocks).  The pivots
// are a and the Schur complement det / a; both must exceed tol.
template <int p>
__device__ __forceinline__ void diag_pivot_pair(double (&d4)[4], double tol, bool& ok, int li,
                                                int lg) {
  constexpr int q = p + 1;
  constexpr int gp = p & 3, ep = p >> 2, gq = q & 3, eq = q >> 2;
  const double a = read_lane(d4[ep], p + 16 * gp);
  const double b = read_lane(d4[eq], p + 16 * gq);  // D[p][q]
  const double c = read_lane(d4[eq], q + 16 * gq);
  const double det = fma(a, c, -b * b);
  ok = ok && a > tol && det > tol * a;
  const double idet = recip(det);
  double zp = rows_bcast<gp>(d4[ep]);  // D[li][p]
  double zq = rows_bcast<gq>(d4[eq]);  // D[li][q]
  double wp[4], wq[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    wp[e] = row_bcast<p>(d4[e]);  // D[p][4 e + lg]
    wq[e] = row_bcast<q>(d4[e]);  // D[q][4 e + lg]
  }
  if (li == p) {
    zp = -1.0;
    zq = 0.0;
  }
  if (li == q) {
    zp = 0.0;
    zq = -1.0;
  }
  // -(z_i B^{-1})
  const double sp = -idet * fma(zp, c, -zq * b);
  const double sq = -idet * fma(zq, a, -zp * b);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool cp = 4 * e + lg == p, cq = 4 * e + lg == q;
    const double x = (li == p || li == q || cp || cq) ? 0.0 : d4[e];
    const double up = cp ? -1.0 : (cq ? 0.0 : wp[e]);
    const double uq = cq ? -1.0 : (cp ? 0.0 : wq[e]);
    d4[e] = fma(sp, up, fma(sq, uq, x));
  }
}

// All pivots p < nbv of the block: pairs while both are pivots, then one.
template <int p>
__device__ __forceinline__ void diag_pivots(double (&d4)[4], int nbv, double tol, bool& ok, int li,
                                            int lg) {
  if constexpr (p < 16) {
    if (p + 1 < nbv) {  // uniform
      diag_pivot_pair<p>(d4, tol, ok, li, lg);
      diag_pivots<p + 2>(d4, nbv, tol, ok, li, lg);
    } else if (p < nbv) {
      diag_pivot<p>(d4, nbv, tol, ok, li, lg);
    }
  }
}

// The matrix lives in registers as 16 x 16 tiles (r, c), c <= r, of the
// lower triangle in the f64 MFMA accumulator layout (element e of lane l is
// (16 r + 4 e + l / 16, 16 c + l % 16)); waves 1..3 own whole tile rows.
// With B the pivots of block b, D = A_BB and Z = A_{:,B} with its rows in B
// replaced by -I, sweeping B is A <- A_{\B} - Y Z^T with Y = Z D^{-1}, where
// A_{\B} has the rows and columns in B zeroed; the columns in B then hold Y
// and the diagonal tile the swept D.
// Two-stage pipeline, one barrier per phase t = 1 .. nblk + 1:
//  * wave 0 takes diagonal tile (b, b), b = t - 1 (handed over by its row
//    owner), applies block b - 1 to it, sweeps its pivots in registers and
//    publishes D^{-1}, the tile's Y rows, its -I panel rows and the swept
//    tile;
//  * waves 1..3 apply block a = t - 2 to their tiles (each forms Y for its
//    own rows on the MFMA), write the panel column of block t - 1 and hand
//    diagonal tile (t, t) to wave 0.
// So the pivot latency chain of one block overlaps the rank-16 update of the
// previous one.  Padding rows and columns (index >= P) are zero throughout.
// solve_only: only the augmented row npiv is wanted (the GGN direction), so
// tiles whose rows are all pivoted -- the part of the inverse that no later
// pivot reads -- are not updated and their Y is not formed.
constexpr int kSweepWaves = 4;

// Orders LDS traffic between the lanes of one wave (a wave executes its LDS
// operations in order, so no s_barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile rows -> update waves 1..3: greedy, largest row (r + 1 tiles) first, to
// the least loaded wave.
__host__ __device__ constexpr int sweep_row_owner(int R, int r) {
  int load[3] = {0, 0, 0}, owner = 0;
  for (int row = R - 1; row >= 0; --row) {
    int w = 0;
    for (int k = 1; k < 3; ++k)
      if (load[k] < load[w]) w = k;
    load[w] += row + 1;
    if (row == r) owner = w + 1;
  }
  return owner;
}
__host__ __device__ constexpr int sweep_tile_row(int t) {
  int r = 0;
  while (t > r) {
    t -= r + 1;
    ++r;
  }
  return r;
}
__host__ __device__ constexpr int sweep_tile_col(int t) {
  return t - sweep_tile_row(t) * (sweep_tile_row(t) + 1) / 2;
}
// register slot of tile t in its owner's array; the owner's slot count
template <int R>
__host__ __device__ constexpr int sweep_slot(int t) {
  int s = 0;
  const int w = sweep_row_owner(R, sweep_tile_row(t));
  for (int u = 0; u < t; ++u)
    if (sweep_row_owner(R, sweep_tile_row(u)) == w) ++s;
  return s;
}
template <int R>
__host__ __device__ constexpr int sweep_slots(int w) {
  int s = 0;
  for (int u = 0; u < R * (R + 1) / 2; ++u)
    if (sweep_row_owner(R, sweep_tile_row(u)) == w) ++s;
  return s;
}

// f(std::integral_constant<int, S>{}) for S = B .. E - 1, so that the body
// sees its index as a constant expression.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// acc += A B^T over one 16-wide k block, A = rows of pa, B = rows of pb (row
// stride kSweepLd, k = column).  Step s takes k = 4 (l / 16) + s from lane l,
// so each lane reads its 4 k-values as two 16-byte LDS loads.
__device__ __forceinline__ f64x4 mfma_abt16(const double* __restrict__ pa,
                                            const double* __restrict__ pb, f64x4 acc, int lane) {
  using f64x2 = double __attribute__((ext_vector_type(2)));
  const int i = lane & 15, q = lane >> 4;
  const f64x2* a2 = reinterpret_cast<const f64x2*>(pa + i * kSweepLd + 4 * q);
  const f64x2* b2 = reinterpret_cast<const f64x2*>(pb + i * kSweepLd + 4 * q);
  const f64x2 a01 = a2[0], a23 = a2[1], b01 = b2[0], b23 = b2[1];
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a01[0], b01[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a01[1], b01[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a23[0], b23[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a23[1], b23[1], acc, 0, 0, 0);
  return acc;
}

// -Y = -(Z D^{-1}) for one row tile (Z = 16 panel rows) into 16 rows of `dst`.
__device__ __forceinline__ void sweep_neg_y(const double* __restrict__ zrows,
                                            const double* __restrict__ dinv,
                                            double* __restrict__ dst, int lane) {
  const int li = lane & 15, q = lane >> 4;
  const f64x4 y = mfma_abt16(zrows, dinv, f64x4{0, 0, 0, 0}, lane);
#pragma unroll
  for (int e = 0; e < 4; ++e) dst[(4 * e + q) * kSweepLd + li] = -y[e];
}

struct SweepLds {
  double* pan;    // 2 panels of 16 R rows
  double* ybufw;  // -Y rows formed by the update waves (each its own rows)
  double* ybufp;  // -Y rows of the swept diagonal tiles
  double* dinv;   // 2 x 16 rows
  double* dtin;   // 2 diagonal tiles handed to wave 0
  double* dtout;  // 2 swept diagonal tiles handed back
  double* ysc;    // wave 0's scratch rows
  double* wmax;
  int* diag_ok;  // 2, by block parity
  int pan_stride;
};

// Wave 0.  Tile (b, b) arrives in dtin[b & 1] with blocks < b - 1 applied.
template <int R>
__device__ __forceinline__ bool sweep_pivot_role(const SweepLds& L, int npiv, int lane) {
  constexpr int LD = kSweepLd, TL = 16 * LD;
  const int li = lane & 15, q = lane >> 4;
  const int nblk = (npiv + 15) / 16;
  if (lane == 0) L.wmax[0] = 0.0;
  __syncthreads();  // phase 0: tiles loaded
  double mx = 0.0;
#pragma unroll
  for (int w = 1; w < kSweepWaves; ++w) mx = fmax(mx, L.wmax[w]);
  const double tol = static_cast<double>(npiv) * 0x1.0p-52 * mx;
  bool ok = true;
#pragma unroll 1
  for (int t = 1; t <= nblk + 1; ++t) {
    const int b = t - 1;
    if (b < nblk) {
      const int nbv = min(16, npiv - 16 * b);
      // d4[e] = D[li][4 e + q] = D[4 e + q][li]: the accumulator layout read
      // as rows (the tile is symmetric)
      f64x4 d;
#pragma unroll
      for (int e = 0; e < 4; ++e) d[e] = L.dtin[(b & 1) * TL + (4 * e + q) * LD + li];
      if (b > 0) {
        const double* zb = L.pan + ((b - 1) & 1) * L.pan_stride + 16 * b * LD;
        sweep_neg_y(zb, L.dinv + ((b - 1) & 1) * TL, L.ysc, lane);
        wave_lds_sync();
        d = mfma_abt16(L.ysc, zb, d, lane);
      }
      // panel rows of block b: -I for the pivots, the tile itself otherwise
      double* pb = L.pan + (b & 1) * L.pan_stride + 16 * b * LD;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pb[li * LD + 4 * e + q] = li < nbv ? (li == 4 * e + q ? -1.0 : 0.0) : d[e];
      double d4[4] = {d[0], d[1], d[2], d[3]};
      bool okb = true;
      diag_pivots<0>(d4, nbv, tol, okb, li, q);
      double* di = L.dinv + (b & 1) * TL;
      double* yp = L.ybufp + 16 * b * LD;
      double* dt = L.dtout + (b & 1) * TL;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * e + q;
        di[li * LD + k] = (li < nbv && k < nbv) ? -d4[e] : 0.0;
        yp[li * LD + k] = k < nbv ? -d4[e] : 0.0;  // the columns in B hold Y
        dt[k * LD + li] = d4[e];
      }
      if (lane == 0) L.diag_ok[b & 1] = okb;
    }
    __syncthreads();
    if (b < nblk) ok = L.diag_ok[b & 1] != 0;
    if (!ok) break;
  }
  return ok;
}

// Update wave W: the tile rows r with sweep_row_owner(R, r) == W.
template <int R, int W, typename TO>
__device__ __forceinline__ bool sweep_update_role(const SweepLds& L, const double* __restrict__ M,
                                                  int P, int npiv, bool solve_only, int lane,
                                                  TO* __restrict__ inv_out, int64_t ldo,
                                                  TO* __restrict__ dir_out) {
  constexpr int LD = kSweepLd, TL = 16 * LD, NT = R * (R + 1) / 2;
  constexpr int NS = sweep_slots<R>(W);
  const int li = lane & 15, q = lane >> 4;
  const int nblk = (npiv + 15) / 16;
  f64x4 acc[NS > 0 ? NS : 1];
  // every tile of this wave, with its row r, column c and slot s as constants
  auto tiles = [&](auto&& f) {
    static_for<0, NT>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      if constexpr (sweep_row_owner(R, sweep_tile_row(t)) == W)
        f(std::integral_constant<int, sweep_tile_row(t)>{},
          std::integral_constant<int, sweep_tile_col(t)>{},
          std::integral_constant<int, sweep_slot<R>(t)>{});
    });
  };

  // phase 0: load, diagonal maximum, hand tile (0, 0) to wave 0
  double dmax = 0.0;
  tiles([&](auto rc, auto cc, auto sc) {
    constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
    f64x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * r + 4 * e + q, j = 16 * c + li;
      v[e] = (i < P && j < P) ? M[static_cast<int64_t>(i) * P + j] : 0.0;
      if (i == j && i < npiv) dmax = fmax(dmax, v[e]);
    }
    acc[s] = v;
    if (r == 0 && c == 0)
#pragma unroll
      for (int e = 0; e < 4; ++e) L.dtin[(4 * e + q) * LD + li] = v[e];
  });
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, kWave));
  if (lane == 0) L.wmax[W] = dmax;
  __syncthreads();

  bool ok = true;
#pragma unroll 1
  for (int t = 1; t <= nblk + 1; ++t) {
    const int a = t - 2;  // the block applied in this phase
    const int nba = a >= 0 ? min(16, npiv - 16 * a) : 0;
    const int np = t - 1;  // the panel column written in this phase
    if (a >= 0) {
      const double* za = L.pan + (a & 1) * L.pan_stride;
      const double* da = L.dinv + (a & 1) * TL;
      // -Y of this wave's rows (the pivot rows come from wave 0)
      static_for<0, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        if constexpr (sweep_row_owner(R, r) == W) {
          if (r != a && !(solve_only && r < a))
            sweep_neg_y(za + 16 * r * LD, da, L.ybufw + 16 * r * LD, lane);
        }
      });
      wave_lds_sync();
      tiles([&](auto rc, auto cc, auto sc) {
        constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
        if (solve_only && r < a) return;
        if (r == c) {
          if (r < nblk && (a == r - 1 || a == r)) {
            if (a == r) {  // swept tile comes back: final for blocks <= r
              f64x4 v;
#pragma unroll
              for (int e = 0; e < 4; ++e) v[e] = L.dtout[(r & 1) * TL + (4 * e + q) * LD + li];
              acc[s] = v;
            }
            return;
          }
        }
        f64x4 x = acc[s];
        if (r == a)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (4 * e + q < nba) x[e] = 0.0;  // rows in B
        if (c == a)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (li < nba) x[e] = 0.0;  // columns in B
        const double* y = (r == a ? L.ybufp : L.ybufw) + 16 * r * LD;
        acc[s] = mfma_abt16(y, za + 16 * c * LD, x, lane);
      });
    }
    if (np < nblk) {
      // panel column np (blocks < np applied): rows of the other tiles
      double* pn = L.pan + (np & 1) * L.pan_stride;
      tiles([&](auto rc, auto cc, auto sc) {
        constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
        if (c == np && r > np) {
#pragma unroll
          for (int e = 0; e < 4; ++e) pn[(16 * r + 4 * e + q) * LD + li] = acc[s][e];
        } else if (r == np && c < np) {
#pragma unroll
          for (int e = 0; e < 4; ++e) pn[(16 * c + li) * LD + 4 * e + q] = acc[s][e];
        }
      });
    }
    if (t < nblk) {
      // diagonal tile (t, t), blocks < t - 1 applied, to wave 0
      tiles([&](auto rc, auto cc, auto sc) {
        constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
        if (r == c && r == t)
#pragma unroll
          for (int e = 0; e < 4; ++e) L.dtin[(t & 1) * TL + (4 * e + q) * LD + li] = acc[s][e];
      });
    }
    __syncthreads();
    if (t - 1 < nblk) ok = L.diag_ok[(t - 1) & 1] != 0;
    if (!ok) break;
  }

  if (inv_out != nullptr) {
    if (ok)
      tiles([&](auto rc, auto cc, auto sc) {
        constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = 16 * r + 4 * e + q, j = 16 * c + li;
          if (i < npiv && j <= i) {
            inv_out[i * ldo + j] = static_cast<TO>(-acc[s][e]);
            inv_out[j * ldo + i] = static_cast<TO>(-acc[s][e]);
          }
        }
      });
  } else {
    // the augmented row npiv holds H^{-1} g in columns j < npiv
    tiles([&](auto rc, auto cc, auto sc) {
      constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * r + 4 * e + q, j = 16 * c + li;
        if (i == npiv && j < npiv) dir_out[j] = ok ? static_cast<TO>(-acc[s][e]) : TO(0);
      }
    });
  }
  return ok;
}

template <int R, typename TO>
__device__ __forceinline__ void sweep_matrix(
    const double* __restrict__ M, int P, int npiv, int mode, TO* __restrict__ inv_out, int64_t ldo,
    TO* __restrict__ dir_out, int32_t* status, int fail_code) {
  constexpr int LD = kSweepLd, TL = 16 * LD;
  __shared__ __attribute__((aligned(16))) double pan[2 * 16 * R * LD];
  __shared__ __attribute__((aligned(16))) double ybufw[16 * R * LD];
  __shared__ __attribute__((aligned(16))) double ybufp[16 * R * LD];
  __shared__ __attribute__((aligned(16))) double tiles16[7 * TL];
  __shared__ double wmax[kSweepWaves];
  __shared__ int diag_ok[2];
  const SweepLds L{pan,           ybufw,          ybufp,    tiles16,  tiles16 + 2 * TL,
                   tiles16 + 4 * TL, tiles16 + 6 * TL, wmax, diag_ok, 16 * R * LD};
  const int lane = threadIdx.x & (kWave - 1);
  // the wave index is uniform: readfirstlane lets each wave take its role
  // (and its tiles) as a scalar branch
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const bool solve_only = mode == kSweepDirection;
  TO* inv = mode == kSweepInverse ? inv_out : nullptr;
  bool ok;
  if (wave == 0)
    ok = sweep_pivot_role<R>(L, npiv, lane);
  else if (wave == 1)
    ok = sweep_update_role<R, 1, TO>(L, M, P, npiv, solve_only, lane, inv, ldo, dir_out);
  else if (wave == 2)
    ok = sweep_update_role<R, 2, TO>(L, M, P, npiv, solve_only, lane, inv, ldo, dir_out);
  else
    ok = sweep_update_role<R, 3, TO>(L, M, P, npiv, solve_only, lane, inv, ldo, dir_out);
  if (threadIdx.x == 0 && status) *status = ok ? GNMPPI_OK : fail_code;
}

template <int R, typename TO>
__global__ void __launch_bounds__(kSweepTD * kSweepTD) sweep_kernel(
    const double* __restrict__ M, int P, int npiv, int mode, TO* __restrict__ inv_out, int64_t ldo,
    TO* __restrict__ dir_out, int32_t* status, int fail_code) {
  sweep_matrix<R, TO>(M, P, npiv, mode, inv_out, ldo, dir_out, status, fail_code);
}

// Batched: MODE 0 inverts Gsum into Ginv (status word 0), MODE 1 solves the
// GGN direction from Hsum into dU (status word 1).  One item per instance.
template <int R, int MODE>
__global__ void __launch_bounds__(kSweepTD * kSweepTD) batch_sweep_kernel(
    const BatchInst* __restrict__ inst, BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchInst& b = inst[L.items[w].inst];
    if constexpr (MODE == 0)
      sweep_matrix<R, float>(b.Gsum, b.n, b.n, kSweepInverse, b.Ginv, b.npad, nullptr, b.status,
                             GNMPPI_ERANK);
    else
      sweep_matrix<R, float>(b.Hsum, b.n + 1, b.n, kSweepDirection, nullptr, 0, b.dU,
                             b.status + 1, GNMPPI_ENOTPD);
    __syncthreads();
  }
}

// One workgroup of 4 waves; R = ceil(P / 16) <= 13 for P <= 208.
template <typename TO>
hipError_t launch_sweep(int P, int npiv, int mode, const double* M, TO* inv_out, int64_t ldo,
                        TO* dir_out, int32_t* status, int fail_code, hipStream_t st) {
  const int R = (P + kSweepTD - 1) / kSweepTD;
#define GNM_SWEEP_CASE(RR)                                                                       \
  case RR:                                                                                       \
    hipLaunchKernelGGL((sweep_kernel<RR, TO>), dim3(1), dim3(kSweepTD * kSweepTD), 0, st, M, P,  \
                       npiv, mode, inv_out, ldo, dir_out, status, fail_code);                    \
    break;
  switch (R) {
    GNM_SWEEP_CASE(1) GNM_SWEEP_CASE(2) GNM_SWEEP_CASE(3) GNM_SWEEP_CASE(4) GNM_SWEEP_CASE(5)
    GNM_SWEEP_CASE(6) GNM_SWEEP_CASE(7) GNM_SWEEP_CASE(8) GNM_SWEEP_CASE(9) GNM_SWEEP_CASE(10)
    GNM_SWEEP_CASE(11) GNM_SWEEP_CASE(12) GNM_SWEEP_CASE(13)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_SWEEP_CASE
  return hipGetLastError();
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

// Batched S = sum of the k-slices; tile = row group * ceil(n / 64) + column group.
__global__ void __launch_bounds__(256) batch_reduce_rows_kernel(const BatchInst* __restrict__ inst,
                                                                BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    const int xb = (b.n + 63) / 64;
    reduce_rows_block<float>(b.part, b.nsplit, static_cast<int64_t>(b.m) * b.npad, b.npad, b.m,
                             b.n, 1.0, b.S, b.npad, nullptr, it.tile % xb, it.tile / xb);
  }
}

// ---- [J r0]^T [J r0] with the f64 MFMA ------------------------------------------

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

// Batched [J r0]^T [J r0] partials; tile = row chunk.
template <int NT>
__global__ void __launch_bounds__(256) batch_gram_kernel(const BatchInst* __restrict__ inst,
                                                         BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchItem it = L.items[w];
    const BatchInst& b = inst[it.inst];
    gram_chunk<float, NT>(b.m, b.n, b.J, b.n, b.r0, 1, b.hchunk, b.n + 1, b.hpart, it.tile);
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

// k-split of the BF16 contraction: blocks of 64 kBf16RowTiles rows; aim at
// two blocks per CU with at least four k-steps per block.
static void bf16_split_plan(int m, int K, int& nsplit_out, int& split_len_out) {
  const int row_blocks = (m + 64 * kBf16RowTiles - 1) / (64 * kBf16RowTiles);
  const int ksteps = (K + 31) / 32;
  int nsplit = (768 + row_blocks - 1) / row_blocks;
  const int max_split = ksteps / 4 > 1 ? ksteps / 4 : 1;
  if (nsplit > max_split) nsplit = max_split;
  if (nsplit < 1) nsplit = 1;
  const int steps_per_split = (ksteps + nsplit - 1) / nsplit;
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
  if (dtype == GNMPPI_F32) bf16_split_plan(m, K, ns_b, sl_b);
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
    bf16_split_plan(m, K, p.nsplit, p.split_len);
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
                     row0, pl.npad, n, n, 0.0, Gsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  (void)K;
  (void)W;
  (void)ldw;
  return launch_sweep<T>(n, n, kSweepInverse, Gsum, Ginv, pl.npad, nullptr, status, GNMPPI_ERANK,
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
                     split_stride, 0, g.P, g.P, n, lm_lambda, Hsum);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == GNMPPI_F32)
    return launch_sweep<float>(g.P, n, kSweepDirection, Hsum, nullptr, 0, static_cast<float*>(dU),
                               status, GNMPPI_ENOTPD, st);
  return launch_sweep<double>(g.P, n, kSweepDirection, Hsum, nullptr, 0, static_cast<double*>(dU),
                              status, GNMPPI_ENOTPD, st);
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
#define GNM_BS_CASE(RR)                                                                         \
  case RR:                                                                                      \
    if (mode == 0)                                                                              \
      hipLaunchKernelGGL((batch_sweep_kernel<RR, 0>), dim3(L.blocks), dim3(kSweepTD * kSweepTD), \
                         0, st, inst, L);                                                       \
    else                                                                                        \
      hipLaunchKernelGGL((batch_sweep_kernel<RR, 1>), dim3(L.blocks), dim3(kSweepTD * kSweepTD), \
                         0, st, inst, L);                                                       \
    break;
  switch (R) {
    GNM_BS_CASE(1) GNM_BS_CASE(2) GNM_BS_CASE(3) GNM_BS_CASE(4) GNM_BS_CASE(5) GNM_BS_CASE(6)
    GNM_BS_CASE(7) GNM_BS_CASE(8) GNM_BS_CASE(9) GNM_BS_CASE(10) GNM_BS_CASE(11)
    default:
      return hipErrorInvalidValue;
  }
#undef GNM_BS_CASE
  return hipGetLastError();
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
