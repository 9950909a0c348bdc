// Dense n x n algebra of the Jacobian reconstruction (Eq. (10)) and of the
// GGN step (Eq. (13)), all in double precision:
//
//  * sweep_kernel    -- one workgroup factors an SPD matrix held as a packed
//                       lower triangle in LDS (n <= 192: 149 KB of the 160 KB
//                       per CU) with the symmetric sweep operator, i.e.
//                       Gauss-Jordan elimination without pivoting, which for
//                       an SPD matrix has the Cholesky pivots.  Sweeping
//                       pivots 0..n-1 of [[H, g], [g^T, c]] leaves -H^{-1} in
//                       the leading block and H^{-1} g in the last row, so
//                       the same kernel yields G^{-1} for the LS Jacobian and
//                       the GGN direction -(H^{-1} g) with no triangular
//                       solves.  A pivot at or below n 2^-52 max diag marks
//                       the matrix as not positive definite.
//  * jac_apply_kernel -- J = S G^{-1} (LS) or J = S / (K sigma^2) (MC); it
//                       also adds up the k-split partial sums of S.
//  * gram_kernel     -- lower-triangular tiles of [J r0]^T [J r0] over a
//                       chunk of rows, in double (products of float inputs
//                       are exact in double).
#include "common.hpp"
#include "launch.hpp"

namespace gnm {

hipError_t launch_jac_contract(int dtype, int m, int n, int rows, int K, const void* R,
                               int64_t ldr, const void* r0, const void* W, int64_t ldw,
                               int nsplit, int split_len, void* part, int npad, hipStream_t st);

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

enum SweepOut { kSweepInverse = 0, kSweepDirection = 1 };

// part: nsplit partial sums, each a row-major matrix with leading dimension
// ldp, the matrix starting at row `row0`; only entries (i, j <= i) are read.
template <typename TP, typename TO>
__global__ void __launch_bounds__(1024) sweep_kernel(const TP* __restrict__ part, int nsplit,
                                                     int64_t split_stride, int row0, int ldp,
                                                     int P, int npiv, double diag_shift, int mode,
                                                     double* __restrict__ inv_out,
                                                     TO* __restrict__ dir_out,
                                                     int32_t* status, int fail_code) {
  __shared__ double A[kMaxSweepDim * (kMaxSweepDim + 1) / 2];
  __shared__ double colv[kMaxSweepDim];
  __shared__ double tol_s;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int nty = blockDim.x >> 5;
  for (int i = ty; i < P; i += nty)
    for (int j = tx; j <= i; j += 32) {
      double s = 0;
      for (int sp = 0; sp < nsplit; ++sp)
        s += static_cast<double>(part[sp * split_stride + static_cast<int64_t>(row0 + i) * ldp + j]);
      if (i == j && i < npiv) s += diag_shift;
      A[tri(i, j)] = s;
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0;
    for (int i = 0; i < npiv; ++i) mx = fmax(mx, A[tri(i, i)]);
    tol_s = static_cast<double>(npiv) * 0x1.0p-52 * mx;
  }
  __syncthreads();
  const double tol = tol_s;
  bool ok = true;
  for (int p = 0; p < npiv; ++p) {
    for (int i = threadIdx.x; i < P; i += blockDim.x) colv[i] = i >= p ? A[tri(i, p)] : A[tri(p, i)];
    __syncthreads();
    const double d = colv[p];
    if (!(d > tol)) {  // every thread reads the same pivot: uniform exit
      ok = false;
      break;
    }
    const double inv = 1.0 / d;
    for (int i = ty; i < P; i += nty)
      for (int j = tx; j <= i; j += 32) {
        double v;
        if (i == p && j == p)
          v = -inv;
        else if (i == p)
          v = colv[j] * inv;
        else if (j == p)
          v = colv[i] * inv;
        else
          v = A[tri(i, j)] - colv[i] * colv[j] * inv;
        A[tri(i, j)] = v;
      }
    __syncthreads();
  }
  if (mode == kSweepInverse) {
    if (ok)
      for (int i = ty; i < npiv; i += nty)
        for (int j = tx; j < npiv; j += 32)
          inv_out[i * npiv + j] = -(j <= i ? A[tri(i, j)] : A[tri(j, i)]);
  } else {
    for (int j = threadIdx.x; j < npiv; j += blockDim.x)
      dir_out[j] = ok ? static_cast<TO>(-A[tri(npiv, j)]) : TO(0);
  }
  if (threadIdx.x == 0 && status) *status = ok ? GNMPPI_OK : fail_code;
}

// J rows [32 b, 32 b + 32): S summed over the k-split partials, then
// multiplied by G^{-1} (LS) or scaled (MC).
constexpr int kApplyRows = 32;
constexpr int kMaxN = 192;

template <typename T>
__global__ void __launch_bounds__(256) jac_apply_kernel(int m, int n, const T* __restrict__ part,
                                                        int nsplit, int64_t split_stride, int npad,
                                                        const double* __restrict__ Ginv,
                                                        double mc_scale, int method,
                                                        T* __restrict__ J, int64_t ldj) {
  __shared__ double Ss[kApplyRows][kMaxN + 1];
  const int i0 = blockIdx.x * kApplyRows;
  const int tid = threadIdx.x;
  for (int e = tid; e < kApplyRows * n; e += blockDim.x) {
    const int r = e / n, c = e - r * n;
    const int i = i0 + r;
    double s = 0;
    if (i < m)
      for (int sp = 0; sp < nsplit; ++sp)
        s += static_cast<double>(part[sp * split_stride + static_cast<int64_t>(i) * npad + c]);
    Ss[r][c] = s;
  }
  __syncthreads();
  if (method == GNMPPI_JAC_MC) {
    for (int e = tid; e < kApplyRows * n; e += blockDim.x) {
      const int r = e / n, c = e - r * n;
      if (i0 + r < m) J[static_cast<int64_t>(i0 + r) * ldj + c] = static_cast<T>(Ss[r][c] * mc_scale);
    }
    return;
  }
  const int tx = tid & 31, ty = tid >> 5;  // columns tx + 32 q, rows ty + 8 p
  constexpr int QN = kMaxN / 32, PR = kApplyRows / 8;
  double acc[PR][QN];
#pragma unroll
  for (int p = 0; p < PR; ++p)
#pragma unroll
    for (int q = 0; q < QN; ++q) acc[p][q] = 0;
  for (int k = 0; k < n; ++k) {
    double g[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int c = tx + 32 * q;
      g[q] = c < n ? Ginv[k * n + c] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < PR; ++p) {
      const double s = Ss[ty + 8 * p][k];
#pragma unroll
      for (int q = 0; q < QN; ++q) acc[p][q] += s * g[q];
    }
  }
#pragma unroll
  for (int p = 0; p < PR; ++p) {
    const int i = i0 + ty + 8 * p;
    if (i >= m) continue;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int c = tx + 32 * q;
      if (c < n) J[static_cast<int64_t>(i) * ldj + c] = static_cast<T>(acc[p][q]);
    }
  }
}

// Lower-triangular 64x64 tiles of X^T X with X = [J r0] (m x (n+1)), over the
// rows of one chunk.  grid.x enumerates tile pairs (ta >= tb), grid.y chunks.
constexpr int kGramTile = 64;
constexpr int kGramSub = 32;

template <typename T>
__global__ void __launch_bounds__(256) gram_kernel(int m, int n, const T* __restrict__ J,
                                                   int64_t ldj, const T* __restrict__ r0,
                                                   int64_t inc, int chunk,
                                                   double* __restrict__ part, int P) {
  __shared__ double Xa[kGramSub][kGramTile + 1];
  __shared__ double Xb[kGramSub][kGramTile + 1];
  int ta = 0, rem = blockIdx.x;
  while (rem > ta) {
    rem -= ta + 1;
    ++ta;
  }
  const int tb = rem;
  const int a0 = ta * kGramTile, b0 = tb * kGramTile;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int ibeg = blockIdx.y * chunk, iend = min(m, ibeg + chunk);
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0;
  auto xval = [&](int i, int c) -> double {
    if (i >= iend || c > n) return 0.0;
    return c < n ? static_cast<double>(J[static_cast<int64_t>(i) * ldj + c])
                 : static_cast<double>(r0[static_cast<int64_t>(i) * inc]);
  };
  for (int s0 = ibeg; s0 < iend; s0 += kGramSub) {
    for (int e = tid; e < kGramSub * kGramTile; e += blockDim.x) {
      const int rr = e / kGramTile, cc = e - rr * kGramTile;
      Xa[rr][cc] = xval(s0 + rr, a0 + cc);
      Xb[rr][cc] = xval(s0 + rr, b0 + cc);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kGramSub; ++rr) {
      double xa[4], xb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xa[u] = Xa[rr][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) xb[v] = Xb[rr][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += xa[u] * xb[v];
    }
    __syncthreads();
  }
  double* out = part + static_cast<int64_t>(blockIdx.y) * P * P;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int a = a0 + ty + 16 * u;
    if (a >= P) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = b0 + tx + 16 * v;
      if (b < P && b <= a) out[static_cast<int64_t>(a) * P + b] = acc[u][v];
    }
  }
}

__global__ void set_status_kernel(int32_t* status, int32_t value) { *status = value; }

}  // namespace

JacPlan jacobian_plan(int dtype, int m, int n, int K, int method) {
  JacPlan p{};
  const int esz = dtype == GNMPPI_F32 ? 4 : 8;
  const int step = dtype == GNMPPI_F32 ? 32 : 16;
  p.ncol_tiles = (n + 15) / 16;
  p.npad = 16 * p.ncol_tiles;
  p.rows = m + (method == GNMPPI_JAC_LS ? n : 0);
  const int waves_per_split = (p.rows + 15) / 16;
  const int ksteps = (K + step - 1) / step;
  int nsplit = (1536 + waves_per_split - 1) / waves_per_split;
  const int max_split = ksteps / 2 > 1 ? ksteps / 2 : 1;
  if (nsplit > max_split) nsplit = max_split;
  if (nsplit < 1) nsplit = 1;
  const int steps_per_split = (ksteps + nsplit - 1) / nsplit;
  p.nsplit = (ksteps + steps_per_split - 1) / steps_per_split;
  p.split_len = steps_per_split * step;
  p.part_bytes = align_up(static_cast<size_t>(p.nsplit) * p.rows * p.npad * esz);
  p.ginv_off = p.part_bytes;
  p.total = p.part_bytes + align_up(static_cast<size_t>(n) * n * 8);
  return p;
}

hipError_t launch_jacobian(int dtype, int m, int n, int K, const void* R, int64_t ldr,
                           const void* r0, const void* W, int64_t ldw, int method, double sigma2,
                           void* J, int64_t ldj, void* work, int32_t* status, hipStream_t st) {
  const JacPlan pl = jacobian_plan(dtype, m, n, K, method);
  char* wk = static_cast<char*>(work);
  hipError_t e = launch_jac_contract(dtype, m, n, pl.rows, K, R, ldr, r0, W, ldw, pl.nsplit,
                                     pl.split_len, wk, pl.npad, st);
  if (e != hipSuccess) return e;
  const int64_t split_stride = static_cast<int64_t>(pl.rows) * pl.npad;
  double* Ginv = reinterpret_cast<double*>(wk + pl.ginv_off);
  if (method == GNMPPI_JAC_LS) {
    if (dtype == GNMPPI_F32)
      hipLaunchKernelGGL((sweep_kernel<float, float>), dim3(1), dim3(1024), 0, st,
                         reinterpret_cast<const float*>(wk), pl.nsplit, split_stride, m, pl.npad,
                         n, n, 0.0, static_cast<int>(kSweepInverse), Ginv,
                         static_cast<float*>(nullptr), status, GNMPPI_ERANK);
    else
      hipLaunchKernelGGL((sweep_kernel<double, double>), dim3(1), dim3(1024), 0, st,
                         reinterpret_cast<const double*>(wk), pl.nsplit, split_stride, m, pl.npad,
                         n, n, 0.0, static_cast<int>(kSweepInverse), Ginv,
                         static_cast<double*>(nullptr), status, GNMPPI_ERANK);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const double mc_scale = 1.0 / (static_cast<double>(K) * sigma2);
  dim3 grid((m + kApplyRows - 1) / kApplyRows);
  if (dtype == GNMPPI_F32)
    hipLaunchKernelGGL(jac_apply_kernel<float>, grid, dim3(256), 0, st, m, n,
                       reinterpret_cast<const float*>(wk), pl.nsplit, split_stride, pl.npad,
                       Ginv, mc_scale, method, static_cast<float*>(J), ldj);
  else
    hipLaunchKernelGGL(jac_apply_kernel<double>, grid, dim3(256), 0, st, m, n,
                       reinterpret_cast<const double*>(wk), pl.nsplit, split_stride, pl.npad,
                       Ginv, mc_scale, method, static_cast<double*>(J), ldj);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (method == GNMPPI_JAC_MC && status) {
    // MC has no factorisation that can fail; report success in stream order.
    hipLaunchKernelGGL(set_status_kernel, dim3(1), dim3(1), 0, st, status, GNMPPI_OK);
    e = hipGetLastError();
  }
  return e;
}

GgnPlan ggn_plan(int dtype, int m, int n) {
  (void)dtype;
  GgnPlan g{};
  g.P = n + 1;
  g.tiles = (g.P + kGramTile - 1) / kGramTile;
  const int pairs = g.tiles * (g.tiles + 1) / 2;
  int nsplit = (128 + pairs - 1) / pairs;
  if (nsplit > 24) nsplit = 24;
  int chunk = (m + nsplit - 1) / nsplit;
  chunk = (chunk + kGramSub - 1) / kGramSub * kGramSub;
  g.chunk = chunk;
  g.nsplit = (m + chunk - 1) / chunk;
  g.total = align_up(static_cast<size_t>(g.nsplit) * g.P * g.P * 8);
  return g;
}

hipError_t launch_ggn(int dtype, int m, int n, const void* J, int64_t ldj, const void* r0,
                      int64_t inc_r0, double lm_lambda, void* dU, void* work, int32_t* status,
                      hipStream_t st) {
  const GgnPlan g = ggn_plan(dtype, m, n);
  double* part = static_cast<double*>(work);
  const int pairs = g.tiles * (g.tiles + 1) / 2;
  dim3 grid(pairs, g.nsplit);
  if (dtype == GNMPPI_F32)
    hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(256), 0, st, m, n,
                       static_cast<const float*>(J), ldj, static_cast<const float*>(r0), inc_r0,
                       g.chunk, part, g.P);
  else
    hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, st, m, n,
                       static_cast<const double*>(J), ldj, static_cast<const double*>(r0),
                       inc_r0, g.chunk, part, g.P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t split_stride = static_cast<int64_t>(g.P) * g.P;
  if (dtype == GNMPPI_F32)
    hipLaunchKernelGGL((sweep_kernel<double, float>), dim3(1), dim3(1024), 0, st, part, g.nsplit,
                       split_stride, 0, g.P, g.P, n, lm_lambda, static_cast<int>(kSweepDirection),
                       static_cast<double*>(nullptr), static_cast<float*>(dU), status,
                       GNMPPI_ENOTPD);
  else
    hipLaunchKernelGGL((sweep_kernel<double, double>), dim3(1), dim3(1024), 0, st, part,
                       g.nsplit, split_stride, 0, g.P, g.P, n, lm_lambda,
                       static_cast<int>(kSweepDirection), static_cast<double*>(nullptr),
                       static_cast<double*>(dU), status, GNMPPI_ENOTPD);
  return hipGetLastError();
}

}  // namespace gnm
