// Warm-start network kernels: a three-layer perceptron I -> H -> H -> O with
// GELU hidden activations, bfloat16 weights and float32 accumulation, its
// squared-error loss, backpropagation and the Adam update.  (The network is
// an extension around Alg. 1: GN-MPPI starts from its proposal instead of
// from zero.)
//
// Every matrix product runs on v_mfma_f32_16x16x32_bf16: both operands are
// rounded to bfloat16 where they are loaded, products are summed in float32.
// One strided GEMM kernel covers the forward products (activations x W^T),
// the input gradients (dZ x W) and the weight gradients (dZ^T x A): operand
// element (i, k) sits at base + i * row_stride + k * k_stride.  The layer
// epilogues are fused: bias, bias + GELU (keeping the pre-activation for the
// backward pass), or the GELU derivative.
//
// Parameter layout (flat, bfloat16 for compute, float32 master copy for
// Adam): W1 (H x I), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O).
#include <cmath>

#include "common.hpp"
#include "launch.hpp"

namespace gnm {
namespace {

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x4 = float __attribute__((ext_vector_type(4)));

enum MlpEpi { kEpiPlain = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluGrad = 3 };

struct MlpGemm {
  int M, N, K;  // C is M x N, contraction over K
  const void* A;
  int64_t a_row, a_k;  // A(i, k) = A[i a_row + k a_k]
  const void* B;
  int64_t b_col, b_k;  // B(j, k) = B[j b_col + k b_k]
  float* C;
  int64_t ldc;
  const __bf16* bias;  // per output column
  float* pre;          // pre-activation (written by kEpiBiasGelu, read by kEpiGeluGrad), ld = ldc
};

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__bf16 v) { return static_cast<float>(v); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Block = 4 waves, a 64 x 64 output tile; wave w owns rows 16 w .. 16 w + 15
// and four 16-column MFMA tiles.  Lane (r16, kq) supplies A[r16][8 kq + e]
// and B[8 kq + e][r16]; accumulator j is C[4 kq + j][r16].
template <typename TA, typename TB, int EPI>
__global__ void __launch_bounds__(256) mlp_gemm_kernel(MlpGemm g) {
  constexpr int NT = 4;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r16 = lane & 15, kq = lane >> 4;
  const int row0 = blockIdx.y * 64 + wave * 16;
  const int col0 = blockIdx.x * 64;
  const TA* A = static_cast<const TA*>(g.A);
  const TB* B = static_cast<const TB*>(g.B);
  const int arow = row0 + r16;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0, 0, 0, 0};
  if (row0 < g.M) {
    for (int k0 = 0; k0 < g.K; k0 += 32) {
      const int kl = k0 + 8 * kq;
      bf16x8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool ok = arow < g.M && kl + e < g.K;
        a[e] = static_cast<__bf16>(ok ? to_f32(A[arow * g.a_row + (kl + e) * g.a_k]) : 0.0f);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = col0 + 16 * t + r16;
        bf16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = col < g.N && kl + e < g.K;
          b[e] = static_cast<__bf16>(ok ? to_f32(B[col * g.b_col + (kl + e) * g.b_k]) : 0.0f);
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = row0 + 4 * kq + j;
    if (row >= g.M) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = col0 + 16 * t + r16;
      if (col >= g.N) continue;
      const int64_t o = row * g.ldc + col;
      float v = acc[t][j];
      if constexpr (EPI == kEpiBias) {
        v += static_cast<float>(g.bias[col]);
      } else if constexpr (EPI == kEpiBiasGelu) {
        v += static_cast<float>(g.bias[col]);
        g.pre[o] = v;
        v = gelu(v);
      } else if constexpr (EPI == kEpiGeluGrad) {
        v *= gelu_grad(g.pre[o]);
      }
      g.C[o] = v;
    }
  }
}

template <typename TA, typename TB, int EPI>
hipError_t gemm(const MlpGemm& g, hipStream_t st) {
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL((mlp_gemm_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

// dY = (Y - T) / (B O) and loss = sum (Y - T)^2 / (2 B O): one block, a
// fixed reduction order (reproducible).
__global__ void __launch_bounds__(1024) mlp_loss_kernel(int64_t count, const float* __restrict__ Y,
                                                        const float* __restrict__ T,
                                                        float* __restrict__ dY, float* loss) {
  __shared__ double part[1024 / kWave];
  const double scale = 1.0 / static_cast<double>(count);
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 1024) {
    const float d = Y[i] - T[i];
    dY[i] = static_cast<float>(d * scale);
    s += static_cast<double>(d) * d;
  }
  for (int off = kWave / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 1024 / kWave; ++w) t += part[w];
    if (loss) *loss = static_cast<float>(0.5 * t * scale);
  }
}

// out[j] = sum_i D[i, j] (the bias gradients): 64 columns x 4 row phases per
// block, phases added in a fixed order.
__global__ void __launch_bounds__(256) mlp_colsum_kernel(int M, int N, const float* __restrict__ D,
                                                         float* __restrict__ out) {
  __shared__ float part[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  float s = 0.0f;
  if (c < N)
    for (int i = ph; i < M; i += 4) s += D[static_cast<int64_t>(i) * N + c];
  part[ph][threadIdx.x & 63] = s;
  __syncthreads();
  if (ph == 0 && c < N) out[c] = ((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) +
                                 part[3][threadIdx.x];
}

__global__ void __launch_bounds__(256) mlp_adam_kernel(int64_t count, float* __restrict__ master,
                                                       __bf16* __restrict__ params,
                                                       const float* __restrict__ grad,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       float lr, float beta1, float beta2, float eps,
                                                       float inv_c1, float inv_c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= count) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * g;
  const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = master[i] - lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
  master[i] = p;
  params[i] = static_cast<__bf16>(p);
}

struct MlpLayout {
  int64_t w1, b1, w2, b2, w3, b3, total;
};

MlpLayout mlp_layout(int I, int H, int O) {
  MlpLayout l{};
  l.w1 = 0;
  l.b1 = l.w1 + static_cast<int64_t>(H) * I;
  l.w2 = l.b1 + H;
  l.b2 = l.w2 + static_cast<int64_t>(H) * H;
  l.w3 = l.b2 + H;
  l.b3 = l.w3 + static_cast<int64_t>(O) * H;
  l.total = l.b3 + O;
  return l;
}

// Workspace: z1, a1, z2, a2, dz2, dz1 (B x H each), y, dy (B x O).
struct MlpWork {
  float *z1, *a1, *z2, *a2, *dz2, *dz1, *y, *dy;
};

MlpWork mlp_work(void* work, int H, int O, int Bt) {
  float* f = static_cast<float*>(work);
  const int64_t bh = static_cast<int64_t>(Bt) * H, bo = static_cast<int64_t>(Bt) * O;
  MlpWork w{};
  w.z1 = f;
  w.a1 = w.z1 + bh;
  w.z2 = w.a1 + bh;
  w.a2 = w.z2 + bh;
  w.dz2 = w.a2 + bh;
  w.dz1 = w.dz2 + bh;
  w.y = w.dz1 + bh;
  w.dy = w.y + bo;
  return w;
}

}  // namespace

int64_t mlp_param_count(int I, int H, int O) { return mlp_layout(I, H, O).total; }

size_t mlp_workspace_bytes(int H, int O, int Bt) {
  return (static_cast<size_t>(6) * Bt * H + static_cast<size_t>(2) * Bt * O) * sizeof(float);
}

hipError_t launch_mlp_forward(int I, int H, int O, int Bt, const void* params, const float* X,
                              float* Y, void* work, hipStream_t st) {
  const MlpLayout l = mlp_layout(I, H, O);
  const __bf16* P = static_cast<const __bf16*>(params);
  const MlpWork w = mlp_work(work, H, O, Bt);
  hipError_t e;
  // z1 = X W1^T + b1, a1 = gelu(z1)
  e = gemm<float, __bf16, kEpiBiasGelu>(
      MlpGemm{Bt, H, I, X, I, 1, P + l.w1, I, 1, w.a1, H, P + l.b1, w.z1}, st);
  if (e != hipSuccess) return e;
  e = gemm<float, __bf16, kEpiBiasGelu>(
      MlpGemm{Bt, H, H, w.a1, H, 1, P + l.w2, H, 1, w.a2, H, P + l.b2, w.z2}, st);
  if (e != hipSuccess) return e;
  return gemm<float, __bf16, kEpiBias>(
      MlpGemm{Bt, O, H, w.a2, H, 1, P + l.w3, H, 1, Y, O, P + l.b3, nullptr}, st);
}

hipError_t launch_mlp_backward(int I, int H, int O, int Bt, const void* params, const float* X,
                               const float* T, float* loss, float* grad, void* work,
                               hipStream_t st) {
  const MlpLayout l = mlp_layout(I, H, O);
  const __bf16* P = static_cast<const __bf16*>(params);
  const MlpWork w = mlp_work(work, H, O, Bt);
  hipError_t e = launch_mlp_forward(I, H, O, Bt, params, X, w.y, work, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1024), 0, st, static_cast<int64_t>(Bt) * O, w.y,
                     T, w.dy, loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // layer 3: gW3 = dY^T a2, gb3 = sum_b dY, dz2 = (dY W3) * gelu'(z2)
  e = gemm<float, float, kEpiPlain>(
      MlpGemm{O, H, Bt, w.dy, 1, O, w.a2, 1, H, grad + l.w3, H, nullptr, nullptr}, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3((O + 63) / 64), dim3(256), 0, st, Bt, O, w.dy,
                     grad + l.b3);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = gemm<float, __bf16, kEpiGeluGrad>(
      MlpGemm{Bt, H, O, w.dy, O, 1, P + l.w3, 1, H, w.dz2, H, nullptr, w.z2}, st);
  if (e != hipSuccess) return e;
  // layer 2
  e = gemm<float, float, kEpiPlain>(
      MlpGemm{H, H, Bt, w.dz2, 1, H, w.a1, 1, H, grad + l.w2, H, nullptr, nullptr}, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3((H + 63) / 64), dim3(256), 0, st, Bt, H, w.dz2,
                     grad + l.b2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = gemm<float, __bf16, kEpiGeluGrad>(
      MlpGemm{Bt, H, H, w.dz2, H, 1, P + l.w2, 1, H, w.dz1, H, nullptr, w.z1}, st);
  if (e != hipSuccess) return e;
  // layer 1
  e = gemm<float, float, kEpiPlain>(
      MlpGemm{H, I, Bt, w.dz1, 1, H, X, 1, I, grad + l.w1, I, nullptr, nullptr}, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3((H + 63) / 64), dim3(256), 0, st, Bt, H, w.dz1,
                     grad + l.b1);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(int64_t count, float* master, void* params, const float* grad, float* m,
                           float* v, double lr, double beta1, double beta2, double eps, int step,
                           hipStream_t st) {
  const double c1 = 1.0 - std::pow(beta1, step), c2 = 1.0 - std::pow(beta2, step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0,
                     st, count, master, static_cast<__bf16*>(params), grad, m, v,
                     static_cast<float>(lr), static_cast<float>(beta1), static_cast<float>(beta2),
                     static_cast<float>(eps), static_cast<float>(1.0 / c1),
                     static_cast<float>(1.0 / c2));
  return hipGetLastError();
}

}  // namespace gnm
