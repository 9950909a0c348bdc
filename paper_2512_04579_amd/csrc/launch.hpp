// Host-side launchers of the GN-MPPI kernels.  The C ABI (abi.cpp) validates
// arguments and calls these; each launcher only enqueues work on `st`.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gnmppi.h"

namespace gnm {

hipError_t launch_sample(int dtype, int n, int K, double sigma, uint64_t seed,
                         uint64_t stream_id, int antithetic, void* W, int64_t ldw,
                         hipStream_t st);
hipError_t launch_sigma_points(int dtype, int n, double sigma, void* W, int64_t ldw,
                               hipStream_t st);

hipError_t launch_rollout(const gnmppi_problem& p, const void* x0, const void* U,
                          const void* W, int64_t ldw, int K, void* R, int64_t ldr,
                          void* C, void* r0, void* c0, hipStream_t st);
// Sampler and rollout in one launch where the chain's split kernel runs (else
// the sampler, then the rollout): W is written, not read.
hipError_t launch_sample_rollout(const gnmppi_problem& p, const void* x0, const void* U,
                                 double sigma, uint64_t seed, uint64_t stream_id, int antithetic,
                                 void* W, int64_t ldw, int K, void* R, int64_t ldr, void* C,
                                 void* r0, void* c0, hipStream_t st);
// With Rc (L residual vectors of m = N (nx + nu) entries each): r0, c0 <- the
// residuals and cost of the chosen candidate.
hipError_t launch_line_search(const gnmppi_problem& p, const void* x0, void* U,
                              const void* dU, const void* alpha, int L, void* C,
                              double* info, int32_t* status, hipStream_t st,
                              void* Rc = nullptr, void* r0 = nullptr, void* c0 = nullptr);

hipError_t launch_mppi_update(int dtype, int n, int K, const void* C, const void* W,
                              int64_t ldw, double temperature, void* U, void* weights,
                              int32_t* status, hipStream_t st);

// out[y] = A B^T over k in [y split_len, (y+1) split_len) for y < nsplit.
// Rows r < m come from A (minus asub[r] when asub is set), rows m <= r < rows
// from A2; output columns are the ncol rows of B, written up to ocols.  With
// asplit > 1, A is itself a sum of asplit partials asplit_stride apart (added
// in order while loading).  status (optional) is set to GNMPPI_OK by block 0.
template <typename T>
struct ContractArgs {
  int m, rows, ncol, K;
  const T* A;
  int64_t lda;
  const T* asub;
  const T* A2;
  int64_t lda2;
  const T* B;
  int64_t ldb;
  int split_len;
  T* out;
  int64_t ldo;
  int64_t split_stride;
  int ocols;
  int asplit = 1;
  int64_t asplit_stride = 0;
  int32_t* status = nullptr;
};
// Waves per block that share one 16-row output tile of launch_contract and
// split its k-steps between them (the planner sizes k-splits with it).
int contract_kw(size_t elem_size, int ncol);
// launch_contract_bf16: 16-row MFMA tiles per wave (a block covers 64 times
// as many rows) and the planner's target for its blocks per k-slice, for
// BF16x3 (three products per term) and for plain BF16 (one product: each
// staged B fragment then feeds two row tiles, and fewer, longer blocks
// stream R better).
constexpr int kBf16RowTiles = 1;
constexpr int kBf16RowTilesPlain = 2;
constexpr int bf16_row_tiles(int terms) { return terms == 3 ? kBf16RowTiles : kBf16RowTilesPlain; }
// k-steps that the BF16 contraction's A loads run ahead of their use (an
// even number: the loop turns over the A ring and both B buffers together).
constexpr int kBf16Depth = 2;
// Blocks the planner aims at for one BF16 contraction (row blocks x k-slices):
// BF16x3 and plain BF16.
constexpr int kBf16BlockTarget = 768;
constexpr int kBf16BlockTargetPlain = 192;
// The batched contraction (throughput-bound, plenty of blocks) takes two
// row tiles per wave: each staged B fragment then feeds twice the MFMAs.
constexpr int kBatchBf16RowTiles = 2;
hipError_t launch_contract(const ContractArgs<float>& a, int nsplit, hipStream_t st);
hipError_t launch_contract(const ContractArgs<double>& a, int nsplit, hipStream_t st);

// BF16 MFMA contraction S = (R - r0 1^T) W^T (terms = 1 or 3); it reads the
// FP32 W and rounds / splits it on its way into LDS.  with_gram: A also
// holds the n rows of W, so each k-slice (m + n rows) carries G = W W^T
// below S.
hipError_t launch_contract_bf16(int terms, int m, int n, int K, const float* R, int64_t ldr,
                                const float* r0, const float* W, int64_t ldw, int nsplit,
                                int split_len, float* part, int npad, hipStream_t st,
                                bool with_gram = false);
// The terms == 1 path of launch_contract_bf16 (defined in gemm_plain.hip).
hipError_t launch_contract_bf16_plain(int nt, dim3 grid, hipStream_t st, int m, int n, int K,
                                      const float* R, int64_t ldr, const float* r0, const float* W,
                                      int64_t ldw, int split_len, float* part, int npad,
                                      int arows, bool vec);

// Symmetric sweep of an SPD matrix M (P x P, full, double) over its first
// npiv pivots (sweep.hpp): kSweepInverse writes the inverse of the leading
// block into inv_out (ldo), kSweepDirection writes the GGN direction
// -(H^{-1} g) of M = [[H, g], [g^T, c]] into dir_out.  A failed pivot writes
// fail_code to *status (else GNMPPI_OK).  P <= 208.
enum SweepOut { kSweepInverse = 0, kSweepDirection = 1 };
// Direction mode with post != nullptr writes post * y (post: symmetric
// npiv x npiv double, leading dimension ldp) in place of the direction y.
hipError_t launch_sweep(int P, int npiv, int mode, const double* M, float* inv_out, int64_t ldo,
                        float* dir_out, int32_t* status, int fail_code, hipStream_t st,
                        const double* post = nullptr, int64_t ldp = 0);
hipError_t launch_sweep(int P, int npiv, int mode, const double* M, double* inv_out, int64_t ldo,
                        double* dir_out, int32_t* status, int fail_code, hipStream_t st,
                        const double* post = nullptr, int64_t ldp = 0);

// Jacobian reconstruction; `work` holds the GEMM partials, G, G^{-1} and S.
struct JacPlan {
  int nsplit;        // k-splits of the S / G contraction
  int split_len;     // samples per split (a multiple of the MFMA k-step)
  int ncol_tiles;    // 16-column tiles covering n
  int npad;          // 16 * ncol_tiles
  int rows;          // m (+ n for LS)
  size_t part_bytes; // bytes of the partial sums
  size_t gsum_off;   // byte offset of G (n x n double, reduced) in work
  size_t ginv_off;   // byte offset of G^{-1} (n x npad, working precision)
  size_t s_off;      // byte offset of S (m x npad, working precision)
  int gsplit;        // k-splits of the separate G = W W^T contraction
  int gsplit_len;
  size_t gpart_off;  // byte offset of its partial sums (gsplit x n x npad)
  int kpad;          // K rounded up to the BF16 MFMA k-step
  size_t total;      // workspace bytes
};
JacPlan jacobian_plan(int dtype, int m, int n, int K, int method);
hipError_t launch_gram(int dtype, int m, int n, int K, const void* W, int64_t ldw, void* work,
                       int32_t* status, hipStream_t st);
hipError_t launch_jacobian(int dtype, int m, int n, int K, const void* R, int64_t ldr,
                           const void* r0, const void* W, int64_t ldw, int method,
                           double sigma2, void* J, int64_t ldj, void* work,
                           int32_t* status, hipStream_t st);

// The GGN direction for the J of launch_jacobian without forming J; the
// workspace is the Jacobian workspace followed by the GGN workspace.
size_t ggn_direction_bytes(int dtype, int m, int n, int K);
hipError_t launch_ggn_direction(int dtype, int m, int n, int K, const void* R, int64_t ldr,
                                const void* r0, const void* W, int64_t ldw, int method,
                                double sigma2, double lm_lambda, void* dU, void* work,
                                int32_t* status, hipStream_t st);

struct GgnPlan {
  int nsplit;        // row chunks of the J^T J contraction
  int chunk;         // rows per chunk
  int P;             // n + 1 (augmented with r0)
  int tiles;         // 16-wide MFMA tiles covering P
  size_t part_bytes; // bytes of the per-chunk partial sums
  size_t total;      // workspace bytes (partials + reduced matrix)
};
GgnPlan ggn_plan(int dtype, int m, int n);
hipError_t launch_ggn(int dtype, int m, int n, const void* J, int64_t ldj, const void* r0,
                      int64_t inc_r0, double lm_lambda, void* dU, void* work,
                      int32_t* status, hipStream_t st);

// The GGN step with its scratch in the library's fixed device array (no
// workspace argument, no allocation); sizes whose ggn_plan total exceeds
// ggn_noalloc_capacity() are rejected with hipErrorInvalidValue.
size_t ggn_noalloc_capacity();
hipError_t launch_ggn_noalloc(int dtype, int m, int n, const void* J, int64_t ldj, const void* r0,
                              int64_t inc_r0, double lm_lambda, void* dU, int32_t* status,
                              hipStream_t st);

// Batched iteration steps (batch.hpp); each launcher covers one shape class.
struct BatchInst;
struct BatchLaunch;
int batch_sample_tiles(int n, int K);
hipError_t launch_batch_sample(const BatchInst* inst, const BatchLaunch& L, double sigma,
                               uint64_t stream_id, hipStream_t st);
int batch_chain_group(int M);
int batch_rollout_tiles(int M, int K);
size_t batch_rollout_lds(int G, int N);
hipError_t launch_batch_rollout(int G, const BatchInst* inst, const BatchLaunch& L,
                                const gnmppi_problem& shared, int N_max, hipStream_t st);
hipError_t launch_batch_nominal(int G, const BatchInst* inst, const BatchLaunch& L,
                                const gnmppi_problem& shared, int N_max, hipStream_t st);
// Fused rollout + sample contraction (fused.hip): one launch for every mass
// count; item = (instance, block of 128 antithetic pairs); writes the item's
// partial sum of S.
constexpr int kFusedPairs = 128;
hipError_t launch_batch_fused(const BatchInst* inst, const BatchLaunch& L,
                              const gnmppi_problem& shared, hipStream_t st);
hipError_t launch_batch_line_search(int G, const BatchInst* inst, const BatchLaunch& L,
                                    const gnmppi_problem& shared, int n_alpha, int N_max,
                                    hipStream_t st);
int batch_contract_row_blocks(int rows);  // 16-row tiles of the G = W W^T contraction
int batch_bf16_row_blocks(int m);
hipError_t launch_batch_contract(int nt, const BatchInst* inst, const BatchLaunch& L,
                                 hipStream_t st);
hipError_t launch_batch_split_bf16(const BatchInst* inst, const BatchLaunch& L, hipStream_t st);
hipError_t launch_batch_contract_bf16(int nt, const BatchInst* inst, const BatchLaunch& L,
                                      hipStream_t st);
hipError_t launch_batch_reduce_sym(int mode, const BatchInst* inst, const BatchLaunch& L,
                                   double lm_lambda, hipStream_t st);
hipError_t launch_batch_sweep(int mode, int R, const BatchInst* inst, const BatchLaunch& L,
                              hipStream_t st);
hipError_t launch_batch_sweep_mode0(int R, const BatchInst* inst, const BatchLaunch& L,
                                    hipStream_t st);
hipError_t launch_batch_sweep_mode1(int R, const BatchInst* inst, const BatchLaunch& L,
                                    hipStream_t st);
hipError_t launch_batch_reduce_rows(const BatchInst* inst, const BatchLaunch& L, hipStream_t st);
hipError_t launch_batch_gram(int nt, const BatchInst* inst, const BatchLaunch& L, hipStream_t st);

// Warm-start perceptron I -> H -> H -> O (mlp.hip).
int64_t mlp_param_count(int I, int H, int O);
size_t mlp_workspace_bytes(int H, int O, int batch);
hipError_t launch_mlp_forward(int I, int H, int O, int batch, const void* params, const float* X,
                              float* Y, void* work, hipStream_t st);
hipError_t launch_mlp_backward(int I, int H, int O, int batch, const void* params, const float* X,
                               const float* T, float* loss, float* grad, void* work,
                               hipStream_t st);
hipError_t launch_mlp_adam(int64_t count, float* master, void* params, const float* grad, float* m,
                           float* v, double lr, double beta1, double beta2, double eps, int step,
                           hipStream_t st);

}  // namespace gnm
