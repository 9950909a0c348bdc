// Blocked register-resident symmetric sweep (the n x n solves of the
// Jacobian reconstruction, Eq. (10), and of the GGN step, Eq. (13)).
// Device code only; the single-instance launchers for float and double
// output and the batched launchers are compiled in separate translation
// units (sweep_f32.hip, sweep_f64.hip, sweep_batch_inv.hip,
// sweep_batch_dir.hip), one per set of template instantiations.
#pragma once

#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace gnm {
namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));

// ---- blocked register-resident symmetric sweep ------------------------------


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
// (16 r + 4 e + l / 16, 16 c + l % 16)); waves 1 .. kSweepWaves - 1 own whole
// tile rows.
// With B the pivots of block b, D = A_BB and Z = A_{:,B} with its rows in B
// replaced by -I, sweeping B is A <- A_{\B} - Y Z^T with Y = Z D^{-1}, where
// A_{\B} has the rows and columns in B zeroed; the columns in B then hold Y
// and the diagonal tile the swept D.
// Two-stage pipeline, one barrier per phase t = 1 .. nblk + 1:
//  * wave 0 takes diagonal tile (b, b), b = t - 1 (handed over by its row
//    owner), applies block b - 1 to it, sweeps its pivots in registers and
//    publishes D^{-1}, the tile's Y rows, its -I panel rows and the swept
//    tile;
//  * the update waves apply block a = t - 2 to their tiles (each forms Y for its
//    own rows on the MFMA), write the panel column of block t - 1 and hand
//    diagonal tile (t, t) to wave 0.
// So the pivot latency chain of one block overlaps the rank-16 update of the
// previous one.  Padding rows and columns (index >= P) are zero throughout.
// solve_only: only the augmented row npiv is wanted (the GGN direction), so
// tiles whose rows are all pivoted -- the part of the inverse that no later
// pivot reads -- are not updated and their Y is not formed.
constexpr int kSweepWaves = 8;
constexpr int kSweepThreads = kSweepWaves * kWave;

// Orders LDS traffic between the lanes of one wave (a wave executes its LDS
// operations in order, so no s_barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile rows -> update waves 1 .. kSweepWaves - 1: greedy, largest row (r + 1
// tiles) first, to the least loaded wave.
__host__ __device__ constexpr int sweep_row_owner(int R, int r) {
  int load[kSweepWaves - 1] = {}, owner = 0;
  for (int row = R - 1; row >= 0; --row) {
    int w = 0;
    for (int k = 1; k < kSweepWaves - 1; ++k)
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

// -Y^T = -(D^{-1} Z^T) for one row tile (Z = 16 panel rows, D^{-1}
// symmetric) in the accumulator layout: element e of lane l is
// -Y[l % 16][4 e + l / 16].
__device__ __forceinline__ f64x4 sweep_neg_yt(const double* __restrict__ zrows,
                                              const double* __restrict__ dinv, int lane) {
  const f64x4 y = mfma_abt16(dinv, zrows, f64x4{0, 0, 0, 0}, lane);
  return f64x4{-y[0], -y[1], -y[2], -y[3]};
}

// acc - Y Z^T for one tile with -Y^T from sweep_neg_yt: step e takes
// k = 4 e + l / 16, its A operand straight from the registers and its B
// operand Z[l % 16][k] from the 16 rows of pb, so Y never goes through LDS.
__device__ __forceinline__ f64x4 mfma_nyt_zt(const f64x4 nyt, const double* __restrict__ pb,
                                             f64x4 acc, int lane) {
  const double* b = pb + (lane & 15) * kSweepLd + (lane >> 4);
  const double b0 = b[0], b1 = b[4], b2 = b[8], b3 = b[12];
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(nyt[0], b0, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(nyt[1], b1, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(nyt[2], b2, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(nyt[3], b3, acc, 0, 0, 0);
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
  double* wmax;
  int* diag_ok;  // 2, by block parity
  int pan_stride;
};

// Wave 0.  Tile (b, b) arrives in dtin[b & 1] with blocks < b - 1 applied.
// In the last phase it has no pivots and waits for the update waves: it then
// reads one word of every 128-byte line of `warm` (warm_bytes bytes, the
// matrix of the post-multiplication), so that those lines are in this XCD's
// L2 when the epilogue reads them; warm_acc keeps the words so the loads stay.
template <int R>
__device__ __forceinline__ bool sweep_pivot_role(const SweepLds& L, int npiv, int lane,
                                                 const double* warm, int64_t warm_bytes,
                                                 uint32_t& warm_acc) {
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
        // block b - 1 applied with its Y^T kept in registers
        const double* zb = L.pan + ((b - 1) & 1) * L.pan_stride + 16 * b * LD;
        d = mfma_nyt_zt(sweep_neg_yt(zb, L.dinv + ((b - 1) & 1) * TL, lane), zb, d, lane);
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
    } else if (warm != nullptr) {
      const char* base = reinterpret_cast<const char*>(warm);
      constexpr int kLines = 8;  // loads in flight per lane and round
      for (int64_t o0 = static_cast<int64_t>(lane) * 128; o0 < warm_bytes;
           o0 += kLines * kWave * 128) {
        uint32_t v[kLines];
#pragma unroll
        for (int u = 0; u < kLines; ++u) {
          const int64_t o = o0 + static_cast<int64_t>(u) * kWave * 128;
          v[u] = *reinterpret_cast<const uint32_t*>(base + min(o, warm_bytes - 8));
        }
#pragma unroll
        for (int u = 0; u < kLines; ++u) warm_acc ^= v[u];
      }
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
                                                  TO* __restrict__ dir_out, double* ydir) {
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
    // the augmented row npiv holds H^{-1} g in columns j < npiv; with a
    // post-multiplication the direction goes to LDS (ydir) first
    tiles([&](auto rc, auto cc, auto sc) {
      constexpr int r = decltype(rc)::value, c = decltype(cc)::value, s = decltype(sc)::value;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * r + 4 * e + q, j = 16 * c + li;
        if (i == npiv && j < npiv) {
          if (ydir != nullptr)
            ydir[j] = -acc[s][e];
          else
            dir_out[j] = ok ? static_cast<TO>(-acc[s][e]) : TO(0);
        }
      }
    });
  }
  return ok;
}

// Update wave `wave` (W .. kSweepWaves - 1) takes its role with its tiles as
// compile-time constants.
template <int R, int W, typename TO>
__device__ __forceinline__ bool sweep_update_dispatch(int wave, const SweepLds& L,
                                                      const double* __restrict__ M, int P,
                                                      int npiv, bool solve_only, int lane,
                                                      TO* __restrict__ inv_out, int64_t ldo,
                                                      TO* __restrict__ dir_out, double* ydir) {
  if constexpr (W + 1 < kSweepWaves) {
    if (wave != W)
      return sweep_update_dispatch<R, W + 1, TO>(wave, L, M, P, npiv, solve_only, lane, inv_out,
                                                 ldo, dir_out, ydir);
  }
  return sweep_update_role<R, W, TO>(L, M, P, npiv, solve_only, lane, inv_out, ldo, dir_out, ydir);
}

// With post != nullptr (direction mode only) the direction y = -H^{-1} g is
// multiplied by the symmetric npiv x npiv matrix `post` (row-major, leading
// dimension ldp) before it is written: dir_out = post y.
template <int R, typename TO>
__device__ __forceinline__ void sweep_matrix(
    const double* __restrict__ M, int P, int npiv, int mode, TO* __restrict__ inv_out, int64_t ldo,
    TO* __restrict__ dir_out, int32_t* status, int fail_code, const double* __restrict__ post,
    int64_t ldp) {
  constexpr int LD = kSweepLd, TL = 16 * LD;
  __shared__ __attribute__((aligned(16))) double pan[2 * 16 * R * LD];
  __shared__ __attribute__((aligned(16))) double ybufw[16 * R * LD];
  __shared__ __attribute__((aligned(16))) double ybufp[16 * R * LD];
  __shared__ __attribute__((aligned(16))) double tiles16[6 * TL];
  __shared__ double wmax[kSweepWaves];
  __shared__ int diag_ok[2];
  // y with zero padding up to the last index the post-multiplication reads
  constexpr int kYdir = 16 * R + kSweepWaves * kWave;
  __shared__ double ydir[kYdir];
  __shared__ double ypart[kSweepWaves * kWave > 16 * R ? kSweepWaves * kWave : 16 * R];
  const SweepLds L{pan,           ybufw,          ybufp,    tiles16,  tiles16 + 2 * TL,
                   tiles16 + 4 * TL, wmax, diag_ok, 16 * R * LD};
  const int lane = threadIdx.x & (kWave - 1);
  // the wave index is uniform: readfirstlane lets each wave take its role
  // (and its tiles) as a scalar branch
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const bool solve_only = mode == kSweepDirection;
  TO* inv = mode == kSweepInverse ? inv_out : nullptr;
  const bool postmul = solve_only && post != nullptr;
  double* yd = postmul ? ydir : nullptr;
  bool ok;
  uint32_t warm_acc = 0;
  if (wave == 0)
    ok = sweep_pivot_role<R>(L, npiv, lane, postmul ? post : nullptr,
                             static_cast<int64_t>(npiv) * ldp * 8, warm_acc);
  else
    ok = sweep_update_dispatch<R, 1, TO>(wave, L, M, P, npiv, solve_only, lane, inv, ldo, dir_out,
                                         yd);
  if (postmul) {
    // dir_out[i] = sum_j post[j][i] y_j (post is symmetric): thread t owns
    // output i = t % kOut for the columns j = h, h + kGroups, ... with
    // h = t / kOut, so each j is one contiguous row segment across the
    // threads; kBatch loads per thread are issued before their products (one
    // memory round trip per batch), and the kGroups partial sums of an output
    // are added in group order through LDS.  y is zero past npiv, and rows
    // past npiv - 1 are read as row npiv - 1, so the loop needs no branches.
    constexpr int kOut = 16 * R;
    constexpr int kGroups = (kSweepWaves * kWave) / kOut > 0 ? (kSweepWaves * kWave) / kOut : 1;
    constexpr int kPerThread = (kOut + kGroups - 1) / kGroups;
    constexpr int kBatch = kPerThread < 32 ? kPerThread : 32;
    for (int j = npiv + static_cast<int>(threadIdx.x); j < kYdir; j += kSweepWaves * kWave)
      ydir[j] = 0.0;
    __syncthreads();
    const int t = threadIdx.x;
    const int i = t % kOut, h = t / kOut;
    double sum = 0.0;
    if (h < kGroups) {
      const int ic = min(i, npiv - 1);
      const int32_t step = kGroups * static_cast<int32_t>(ldp);
      const int32_t last = (npiv - 1) * static_cast<int32_t>(ldp) + ic;
      int32_t off = h * static_cast<int32_t>(ldp) + ic;
      const double* yh = ydir + h;
#pragma unroll 1
      for (int q0 = 0; q0 < kPerThread; q0 += kBatch) {
        double v[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          v[q] = post[min(off, last)];
          off += step;
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) sum = fma(v[q], yh[kGroups * q], sum);
        yh += kGroups * kBatch;
      }
      ypart[h * kOut + i] = sum;
    }
    __syncthreads();
    // (never true: keeps the warm-up loads of wave 0)
    if (warm_acc == 0x2545F491u && npiv < 0) dir_out[0] = TO(0);
    if (t < npiv) {
      double d = ypart[t];
#pragma unroll
      for (int g = 1; g < kGroups; ++g) d += ypart[g * kOut + t];
      dir_out[t] = ok ? static_cast<TO>(d) : TO(0);
    }
  }
  if (threadIdx.x == 0 && status) *status = ok ? GNMPPI_OK : fail_code;
}

template <int R, typename TO>
__global__ void __launch_bounds__(kSweepThreads) sweep_kernel(
    const double* __restrict__ M, int P, int npiv, int mode, TO* __restrict__ inv_out, int64_t ldo,
    TO* __restrict__ dir_out, int32_t* status, int fail_code, const double* __restrict__ post,
    int64_t ldp) {
  sweep_matrix<R, TO>(M, P, npiv, mode, inv_out, ldo, dir_out, status, fail_code, post, ldp);
}

// Batched: MODE 0 inverts Gsum into Ginv (status word 0: the rank check of
// G), MODE 1 solves (S^T S + lambda G^2) y = -S^T r0 from Hsum and writes the
// GGN direction dU = G y (status word 1).  One item per instance.
template <int R, int MODE>
__global__ void __launch_bounds__(kSweepThreads) batch_sweep_kernel(
    const BatchInst* __restrict__ inst, BatchLaunch L) {
  for (int w = blockIdx.x; w < L.count; w += gridDim.x) {
    const BatchInst& b = inst[L.items[w].inst];
    if constexpr (MODE == 0)
      sweep_matrix<R, float>(b.Gsum, b.n, b.n, kSweepInverse, b.Ginv, b.npad, nullptr, b.status,
                             GNMPPI_ERANK, nullptr, 0);
    else
      sweep_matrix<R, float>(b.Hsum, b.n + 1, b.n, kSweepDirection, nullptr, 0, b.dU,
                             b.status + 1, GNMPPI_ENOTPD, b.Gsum, b.n);
    __syncthreads();
  }
}

}  // namespace
}  // namespace gnm
