/*
 * gnmppi.h -- C ABI of the Gauss-Newton accelerated MPPI hot path
 * (Homburger, Baumgaertner, Diehl, Reuter, arXiv 2512.04579) on AMD Instinct
 * MI355X (gfx950).
 *
 * The library solves the direct single-shooting optimal control problem of
 * Sec. 2: an initial state x0 in R^nx, a control sequence
 * U = [u_0; ...; u_{N-1}] in R^{N nu} stacked time-major, the simulator
 * X = F(x0, U) of Eq. (1), and a cost with the least-squares structure
 * C = Phi(R(x0, U)) of Eq. (4) with Phi(R) = 1/2 ||R||^2.
 *
 * Residual convention: for each step k = 0..N-1 the residual holds nx rows
 * sqrt(2 q) .* (x_{k+1} - x_ref) followed by nu rows sqrt(2 r) .* u_k, so
 * m = N (nx + nu) rows, n = N nu decision variables, and 1/2 ||R||^2 is the
 * quadratic stage-plus-terminal cost of Eq. (2) (terminal weight Q, the
 * constant x_0 term dropped).
 *
 * Conventions shared by every call:
 *  - All array pointers are DEVICE pointers owned by the caller; the library
 *    never allocates or frees memory and keeps no state between calls.
 *  - Element type is uniform per call: GNMPPI_F32 (float) or GNMPPI_F64
 *    (double).  Normal-equation factorisations run in double regardless.
 *  - Matrices over samples are "sample-fastest": element (row i, sample s)
 *    of a matrix with leading dimension ld sits at index i*ld + s.
 *  - Every call only enqueues work on `stream` (a hipStream_t; NULL is the
 *    null stream) and returns without synchronising, so a sequence of calls
 *    can be captured into a HIP graph.  The calls do not issue memsets.
 *  - Host-detectable errors (NULL required pointer, non-positive or
 *    inconsistent size, too small a workspace) return a negative code
 *    synchronously and enqueue nothing.  Numerical failures found on the
 *    device are written to the caller's `int32_t *status` word (0 = ok), which
 *    keeps the calls asynchronous.
 *  - Calls on one stream are ordered; concurrent calls on different streams
 *    must not share output or workspace buffers.
 */
#ifndef GNMPPI_H
#define GNMPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GNMPPI_OK          0
#define GNMPPI_EINVAL     (-1) /* invalid argument (host, synchronous)            */
#define GNMPPI_EHIP       (-2) /* HIP runtime error at launch (host, synchronous) */
#define GNMPPI_ENOTPD     (-3) /* device: normal matrix J^T J + lambda I not PD    */
#define GNMPPI_ERANK      (-4) /* device: perturbations do not span R^n (LS form)  */
#define GNMPPI_ENONFINITE (-5) /* device: no sample / candidate had a finite cost  */
#define GNMPPI_ENOSPACE   (-6) /* workspace smaller than the *_workspace() size    */

/* ---- element types, models, estimators ---------------------------------- */
#define GNMPPI_F32 0
#define GNMPPI_F64 1

/* Problem IV (Sec. 5): d independent double integrators with exact zero-order
 * hold, p+ = p + dt v + dt^2/2 u, v+ = v + dt u; state (p_1..p_d, v_1..v_d),
 * nx = 2d, nu = d, 1 <= d <= 4. */
#define GNMPPI_MODEL_DOUBLE_INTEGRATOR 1
/* Planar chain of M point masses (1 <= M <= 16) joined to a fixed anchor and
 * to each other by zero-rest-length springs with force
 * (k_lin + k_cub |d|^2) d; free masses accelerate by (T_{i+1} - T_i) / mass;
 * the end mass moves with the commanded velocity u (nu = 2) and its velocity
 * slot is set to u after each step; classical RK4 with u held over the step
 * (the discretisation of Problem V).  State (p_1..p_M, v_1..v_M), each a 2-D
 * vector, nx = 4M. */
#define GNMPPI_MODEL_CHAIN 2

/* Jacobian estimators for Eq. (10) (Sec. 4.1).
 * LS: J = (dR W^T)(W W^T)^{-1}, the least-squares fit of the residual
 *     differences dR = R(U + W_s) - R(U) to the perturbations; this is
 *     Eq. (10) with Sigma replaced by the samples' second moment.
 * MC: J = (dR W^T) / (K sigma2), the Monte-Carlo mean of Eq. (10) itself. */
#define GNMPPI_JAC_LS 0
#define GNMPPI_JAC_MC 1
/* Flag for GNMPPI_JAC_LS: G^{-1} is already in `work`, computed from the same
 * W by gnmppi_perturbation_gram (possibly on another stream, ordered before
 * this call by the caller), so only S and J = S G^{-1} are formed; the rank
 * check is then reported in gnmppi_perturbation_gram's status word and this
 * call writes GNMPPI_OK to its own. */
#define GNMPPI_JAC_GRAM_READY 0x100
/* Flags for GNMPPI_F32 (either method): form S = dR W^T on the BF16 MFMA with
 * FP32 accumulation.  BF16 rounds dR and W to bf16 (about 2^-9 relative per
 * product: the "precision split").  BF16X3 splits each operand into hi + lo
 * bf16 parts and sums the three leading products, which keeps FP32-level
 * error (about 1e-6 relative on J at the c2 size) at the BF16 MFMA rate.  G
 * stays on the FP32 contraction.  The two flags are mutually exclusive. */
#define GNMPPI_JAC_BF16 0x200
#define GNMPPI_JAC_BF16X3 0x400
/* Flags for GNMPPI_JAC_LS | GNMPPI_JAC_GRAM_READY that split the call in
 * two, so that a caller needs to order the stream that ran
 * gnmppi_perturbation_gram (which writes only the G region of `work`)
 * before the second half only: S_ONLY forms the
 * k-slice partial sums of S = dR W^T in `work` and writes neither J nor the
 * status word; a later APPLY_ONLY call with the same dtype, m, n, K, work
 * and other method bits forms J = S G^{-1} from them (R and W are not read)
 * and writes GNMPPI_OK to its status word.  The two flags are mutually
 * exclusive. */
#define GNMPPI_JAC_S_ONLY 0x800
#define GNMPPI_JAC_APPLY_ONLY 0x1000

/* Problem data (Sec. 2).  Vectors are device arrays of the problem's dtype. */
typedef struct gnmppi_problem {
  int32_t model;    /* GNMPPI_MODEL_*                                   */
  int32_t dtype;    /* GNMPPI_F32 or GNMPPI_F64                          */
  int32_t nx;       /* state dimension                                   */
  int32_t nu;       /* input dimension                                   */
  int32_t N;        /* horizon (number of steps), >= 1                   */
  int32_t n_masses; /* chain only: M                                     */
  double dt;        /* step length                                       */
  double k_lin;     /* chain only: linear spring constant                */
  double k_cub;     /* chain only: cubic spring constant                 */
  double mass;      /* chain only: mass of each free point mass (> 0)    */
  const void *q;    /* nx entries: diagonal of the state weight Q (>= 0) */
  const void *r;    /* nu entries: diagonal of the input weight R (>= 0) */
  const void *x_ref;/* nx entries: tracking target                       */
} gnmppi_problem;

/* ---- a1: perturbation sampler (Sec. 3, W ~ N(0, sigma^2 I); antithetic
 *      pairs as used for Methods C and D, Sec. 5) -------------------------
 * Fills W (n x K, leading dimension ldw >= K) with sigma * z, z standard
 * normal.  z comes from Philox4x32-10 (Salmon et al., SC'11) with
 * key = (seed low word, seed high word) and
 * counter = (column s, row block b, stream low word, stream high word),
 * followed by Box-Muller:
 *   F32: block b -> rows 4b..4b+3; words (x0,x1) give rows 4b, 4b+1 and
 *        (x2,x3) rows 4b+2, 4b+3, with u1 = ((x>>8)+1) 2^-24 from the first
 *        word and u2 = (x>>8) 2^-24 from the second;
 *   F64: block b -> rows 2b, 2b+1 with u1 = (((x0<<21)|(x1>>11))+1) 2^-53
 *        and u2 = ((x2<<21)|(x3>>11)) 2^-53;
 *   z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
 * With antithetic != 0, K must be even, columns s < K/2 are drawn and
 * column s + K/2 is the exact negation of column s.  `stream_id` selects an
 * independent sequence (e.g. the iteration number).
 * Returns GNMPPI_EINVAL for n < 1, K < 1, ldw < K, odd K with antithetic. */
int gnmppi_sample(int32_t dtype, int32_t n, int32_t K, double sigma,
                  uint64_t seed, uint64_t stream_id, int32_t antithetic,
                  void *W, int64_t ldw, void *stream);

/* Method E (Sec. 5): the deterministic Dirac-mixture (sigma-point) set
 * W = [ +sqrt(n) sigma I, -sqrt(n) sigma I ] with K = 2n columns, whose
 * second moment is exactly sigma^2 I.  ldw >= 2n. */
int gnmppi_sigma_points(int32_t dtype, int32_t n, double sigma, void *W,
                        int64_t ldw, void *stream);

/* ---- a2: rollout, residual and cost (Eqs. (1), (2), (4)) ----------------
 * Single shooting of K perturbed control sequences: column s = 0..K-1 uses
 * U + W[:, s] (W == NULL: every column uses U).  Writes the residual column
 * s to R[i*ldr + s] (i < m; R == NULL skips it: costs only) and
 * C[s] = 1/2 ||R[:, s]||^2 (C == NULL skips the costs: residuals only; R and
 * C may not both be NULL when K > 0).  If c0 != NULL the nominal sequence U itself is
 * rolled out in the same launch: its cost goes to c0[0] and, if r0 != NULL,
 * its residual to r0[0..m-1] (contiguous).  K may be 0 when c0 != NULL.
 * x0: nx entries; U: n entries.  Errors: EINVAL for an unsupported model or
 * size, ldw < K, ldr < K. */
int gnmppi_rollout(const gnmppi_problem *p, const void *x0, const void *U,
                   const void *W, int64_t ldw, int32_t K,
                   void *R, int64_t ldr, void *C,
                   void *r0, void *c0, void *stream);

/* ---- a1 + a2 in one launch ----------------------------------------------
 * gnmppi_sample(dtype, n = N nu, K, sigma, seed, stream_id, antithetic, W,
 * ldw) followed by gnmppi_rollout(p, x0, U, W, ldw, K, R, ldr, C, r0, c0),
 * with the same results bit for bit: W (written, not read) holds the draws
 * and R, C, r0, c0 the rollout of U + W[:, s].  For the chain model with
 * staged controls and residuals wanted (R or r0 non-NULL) each rollout block
 * draws its own columns of W while it stages its controls, so the sampler
 * is not a launch of its own; otherwise the two run one after the other.
 * Errors: those of both calls (K >= 1 here). */
int gnmppi_sample_rollout(const gnmppi_problem *p, const void *x0, const void *U,
                          double sigma, uint64_t seed, uint64_t stream_id,
                          int32_t antithetic, void *W, int64_t ldw, int32_t K,
                          void *R, int64_t ldr, void *C, void *r0, void *c0,
                          void *stream);

/* ---- a3: MPPI update (Eqs. (7), (8)) ------------------------------------
 * U <- U + sum_s w_s W[:, s] / sum_s w_s with w_s = exp(-(C_s - min C)/temperature).
 * The shift by min C cancels in the ratio.  Samples with a NaN or infinite
 * cost get weight 0.  If no cost is finite, U is left unchanged and
 * *status = GNMPPI_ENONFINITE, else *status = 0 (status may be NULL).
 * weights (optional, K entries) receives the normalised w_s.  K <= 32768
 * (F32) or 16384 (F64); temperature > 0. */
int gnmppi_mppi_update(int32_t dtype, int32_t n, int32_t K, const void *C,
                       const void *W, int64_t ldw, double temperature,
                       void *U, void *weights, int32_t *status, void *stream);

/* ---- a4: Jacobian reconstruction (Eq. (10), Sec. 4.1) -------------------
 * R: m x K residuals of the perturbed columns (leading dimension ldr),
 * r0: m nominal residuals, W: n x K perturbations (ldw).  Forms
 * S = (R - r0 1^T) W^T and, for LS, G = W W^T, factors G in double precision
 * and writes J = S G^{-1} (LS) or J = S / (K sigma2) (MC) as an m x n
 * row-major matrix with leading dimension ldj >= n.  For LS, a pivot of G
 * below n * 2^-52 * max diag(G) sets *status = GNMPPI_ERANK and J is left
 * unspecified.  Limits: 1 <= n <= 192.  `work` is device scratch of at least
 * gnmppi_jacobian_workspace(...) bytes, 256-byte aligned. */
size_t gnmppi_jacobian_workspace(int32_t dtype, int32_t m, int32_t n, int32_t K);
int gnmppi_reconstruct_jacobian(int32_t dtype, int32_t m, int32_t n, int32_t K,
                                const void *R, int64_t ldr, const void *r0,
                                const void *W, int64_t ldw, int32_t method,
                                double sigma2, void *J, int64_t ldj,
                                void *work, size_t work_bytes,
                                int32_t *status, void *stream);

/* The W-only half of the LS reconstruction: G = W W^T and its inverse (the
 * second-moment matrix that replaces Sigma in Eq. (10)), written into `work`
 * (the Jacobian workspace, same size rule) for a later
 * gnmppi_reconstruct_jacobian(..., GNMPPI_JAC_LS | GNMPPI_JAC_GRAM_READY, ...)
 * with the same dtype, n, K, W and work.  Because it does not depend on the
 * rollout, it can run concurrently with gnmppi_rollout on a second stream.
 * A pivot below n 2^-52 max diag(G) sets *status = GNMPPI_ERANK. */
int gnmppi_perturbation_gram(int32_t dtype, int32_t m, int32_t n, int32_t K, const void *W,
                             int64_t ldw, void *work, size_t work_bytes, int32_t *status,
                             void *stream);

/* ---- a5: Generalized Gauss-Newton step (Eq. (13), Sec. 4.2) -------------
 * dU = -(J^T J + lm_lambda I)^{-1} J^T r0 for Phi = 1/2 ||.||^2, i.e. the
 * minimiser of the GGN subproblem.  J: m x n row-major (ldj), r0: m entries
 * with stride inc_r0.  J^T J and J^T r0 are accumulated in double precision
 * and the system is solved there by the symmetric sweep operator (no
 * pivoting; for an SPD matrix its pivots are the Cholesky pivots); dU is
 * written in dtype.  A pivot at or below n 2^-52 max_i H_ii sets
 * *status = GNMPPI_ENOTPD and dU = 0.  1 <= n <= 192.
 * `work`: at least gnmppi_ggn_workspace(...) bytes, 256-byte aligned. */
size_t gnmppi_ggn_workspace(int32_t dtype, int32_t m, int32_t n);
int gnmppi_ggn_step(int32_t dtype, int32_t m, int32_t n, const void *J,
                    int64_t ldj, const void *r0, int64_t inc_r0,
                    double lm_lambda, void *dU, void *work, size_t work_bytes,
                    int32_t *status, void *stream);

/* ---- a4 + a5 without forming J (Eqs. (10), (13)) ------------------------
 * The GGN direction of gnmppi_ggn_step for the Jacobian that
 * gnmppi_reconstruct_jacobian(..., method, ...) would form, computed from
 * S = (R - r0 1^T) W^T directly.  With J = S A (LS: A = G^{-1}, G = W W^T;
 * MC: A = I / (K sigma2)) and B = A^{-1}, J^T J + lm_lambda I equals
 * A (S^T S + lm_lambda B^2) A and J^T r0 = A S^T r0, so
 *   dU = B y  with  (S^T S + lm_lambda B^2) y = -S^T r0,
 * the same minimiser of the GGN subproblem up to rounding.  LS solves this
 * system (the normal matrix of [S r0], plus lm_lambda G^2, accumulated in
 * double precision; the sweep of gnmppi_ggn_step; then dU = G y), so the
 * m x n x n product J = S G^{-1} is never formed; G comes out of the same
 * contraction as S (the rows of W appended to those of R - r0 1^T), or,
 * with GNMPPI_JAC_GRAM_READY, from gnmppi_perturbation_gram on the same
 * `work` (which then also reports the rank check of G).  MC forms
 * J = S / (K sigma2) and takes the plain GGN step.
 * Arguments as in gnmppi_reconstruct_jacobian and gnmppi_ggn_step (r0
 * contiguous).  method: GNMPPI_JAC_LS (optionally | GNMPPI_JAC_GRAM_READY)
 * or GNMPPI_JAC_MC, either with GNMPPI_JAC_BF16 or GNMPPI_JAC_BF16X3 (F32).
 * LS also takes GNMPPI_JAC_S_ONLY (only the k-slice partials of the
 * contraction; status not written) and GNMPPI_JAC_APPLY_ONLY (the rest, from
 * those partials, with the same other method bits; R and W not read), so that
 * only the second half needs to wait for gnmppi_perturbation_gram.  A pivot
 * at or below n 2^-52 times the largest diagonal entry of the system sets
 * *status = GNMPPI_ENOTPD and dU = 0 (a rank-deficient W makes S^T S
 * singular).  1 <= n <= 192.  `work`: at least
 * gnmppi_ggn_direction_workspace(...) bytes, 256-byte aligned: the Jacobian
 * workspace (its G region is what gnmppi_perturbation_gram writes) followed
 * by the GGN workspace. */
size_t gnmppi_ggn_direction_workspace(int32_t dtype, int32_t m, int32_t n, int32_t K);
int gnmppi_ggn_direction(int32_t dtype, int32_t m, int32_t n, int32_t K,
                         const void *R, int64_t ldr, const void *r0,
                         const void *W, int64_t ldw, int32_t method,
                         double sigma2, double lm_lambda, void *dU,
                         void *work, size_t work_bytes, int32_t *status,
                         void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture that may not call hipMalloc, tight serving loops, harnesses that
 * forbid allocation: gnmppi_ggn_step with no `work` argument.  Its scratch
 * (the J^T J chunk partials and the reduced normal matrix) is an 8 MiB array
 * in device memory defined by the library; each GPU the library runs on
 * holds its own copy until the process ends.  The call allocates nothing.
 * Sizes with gnmppi_ggn_workspace(dtype, m, n) > 8388608 bytes (8 MiB; e.g.
 * n = 100 allows m up to 25856, n = 192 up to 6912) return
 * GNMPPI_ENOSPACE and enqueue nothing.  Every call on one GPU uses that GPU's
 * one array, so calls that overlap in time on one GPU (different streams or
 * threads) race: the caller must order them.  Arguments, results and the
 * status word are those of gnmppi_ggn_step. */
int gnmppi_ggn_step_noalloc(int32_t dtype, int32_t m, int32_t n, const void *J,
                            int64_t ldj, const void *r0, int64_t inc_r0,
                            double lm_lambda, void *dU, int32_t *status,
                            void *stream);

/* ---- a6: parallel line search and update (Eqs. (14), (15); Alg. 1) ------
 * Rolls out the L candidates U + alpha[j] dU in one launch (costs only),
 * picks j* = the first index of the smallest finite cost, and applies
 * U <- U + alpha[j*] dU in place.  alpha: L step lengths (device, dtype),
 * 1 <= L <= 64.  C (optional): the L candidate costs.  info (optional,
 * device double[3]): {alpha[j*], C_j*, j*}.  status (optional, device
 * int32): GNMPPI_OK, or GNMPPI_ENONFINITE if no candidate cost is finite --
 * then U is unchanged and info = {0, NaN, -1}. */
int gnmppi_line_search(const gnmppi_problem *p, const void *x0, void *U,
                       const void *dU, const void *alpha, int32_t L, void *C,
                       double *info, int32_t *status, void *stream);

/* gnmppi_line_search that also returns the nominal rollout of the updated
 * controls, the r0 and c0 that the next iteration's rollout (Eqs. (1), (2),
 * (4)) would produce for column K: the chosen candidate U + alpha[j*] dU IS
 * the next iterate, so its residual rows (kept while the candidates roll out)
 * and its cost are those values, and that rollout can leave out the nominal
 * column.  Rc: device scratch for the L candidates' residual vectors, L * m
 * entries of dtype, m = N (nx + nu); r0: m entries (out); c0: one entry
 * (out, 1/2 ||r0||^2, summed in the line search's order).  If no candidate
 * cost is finite, U, r0 and c0 are left unchanged.  The rows follow R's
 * order; their values are bitwise those of the rollout for the same
 * controls.  Null Rc, r0 or c0: GNMPPI_EINVAL.  Everything else as
 * gnmppi_line_search. */
int gnmppi_line_search_nominal(const gnmppi_problem *p, const void *x0, void *U,
                               const void *dU, const void *alpha, int32_t L,
                               void *C, double *info, int32_t *status, void *Rc,
                               void *r0, void *c0, void *stream);

/* ---- batched iterations ----------------------------------------------------
 *
 * Many independent chain MPC instances of uneven size solved together: one
 * GN-MPPI iteration (Alg. 1: sample, rollout, Jacobian reconstruction of
 * Eq. (10) in the LS form with the BF16x3 sample contraction, GGN step of
 * Eq. (13) in FP64, line search of Eqs. (14)-(15)) for every instance is
 * enqueued by one call, as a few persistent launches per step (one per
 * shape class), so that the whole iteration can be captured in a HIP graph.
 *
 * `shared`: the chain model parameters common to all instances (model =
 * GNMPPI_MODEL_CHAIN, dtype = GNMPPI_F32, dt, k_lin, k_cub, mass; the size
 * fields and q / r / x_ref are ignored).  Instance b: 3 <= n_masses <= 16,
 * 1 <= N <= 80, K even with K / 2 >= 2 N (antithetic pairs must span the
 * decisions), K <= 65536; device float32 x0 (4M), q (4M), r (2), x_ref (4M)
 * and U (2N, the iterate, updated in place); status (3 int32: Jacobian rank,
 * GGN positive definiteness and line search, as the single-instance calls
 * report them) and
 * info (3 doubles: alpha*, C*, j* of the last line search).  Instance b
 * draws its perturbations from Philox key seed + b and stream id = the
 * iteration index, exactly as gnmppi_sample with that seed would.
 *
 * The workspace (gnmppi_batch_workspace bytes, 256-byte aligned, owned by
 * the caller) holds the per-instance W, R, S, J and solve buffers and the
 * work tables; gnmppi_batch_prepare fills the tables (synchronous copies,
 * call it once, outside graph capture).  gnmppi_batch_iteration only
 * enqueues kernels on `stream` and must be given the same instances,
 * settings and tuning as the prepare call.  The tuning fields only change
 * launch shapes and k-slices (0 = default); any value gives a correct
 * result.  Errors: GNMPPI_EINVAL for a rejected argument, GNMPPI_ENOSPACE
 * for a short workspace. */
typedef struct {
  int32_t n_masses, N, K, reserved;
  const void *x0, *q, *r, *x_ref;
  void *U;
  int32_t *status;
  double *info;
} gnmppi_batch_instance;

typedef struct {
  uint64_t seed;     /* instance b uses Philox key seed + b */
  double gamma;      /* line-search ratio, 0 < gamma < 1 */
  int32_t n_alpha;   /* line-search candidates gamma^j, 1 <= n_alpha <= 64 */
  int32_t reserved;
  double lm_lambda;  /* lambda added to the diagonal of J^T J (>= 0) */
} gnmppi_batch_settings;

typedef struct {
  int32_t rollout_blocks_per_cu;   /* persistent grid of the rollout */
  int32_t contract_blocks_per_cu;  /* persistent grid of S = dR W^T */
  int32_t contract_ksplit;         /* k-slices of S per instance */
  int32_t small_blocks_per_cu;     /* persistent grid of the other steps */
  int32_t rollout_mode;            /* 1: lane-group rollout storing the
                                      residuals, then the BF16x3 contraction;
                                      2: rollout fused with the contraction
                                      (one lane per sample, pair differences
                                      contracted on the MFMA, no residuals in
                                      HBM; the contraction tuning fields do
                                      not apply); 0: the default (2) */
} gnmppi_batch_tuning;

size_t gnmppi_batch_workspace(const gnmppi_problem *shared, int32_t count,
                              const gnmppi_batch_instance *inst,
                              const gnmppi_batch_settings *settings,
                              const gnmppi_batch_tuning *tuning);
int gnmppi_batch_prepare(const gnmppi_problem *shared, int32_t count,
                         const gnmppi_batch_instance *inst, const gnmppi_batch_settings *settings,
                         const gnmppi_batch_tuning *tuning, void *work, size_t work_bytes);
int gnmppi_batch_iteration(const gnmppi_problem *shared, int32_t count,
                           const gnmppi_batch_instance *inst,
                           const gnmppi_batch_settings *settings,
                           const gnmppi_batch_tuning *tuning, void *work, size_t work_bytes,
                           int32_t it, double sigma, void *stream);

/* ---- learned warm start ----------------------------------------------------
 *
 * Not part of the paper's method: a perceptron proposes the initial control
 * sequence U0(x0) from which Alg. 1 starts (GN-MPPI from zero remains the
 * fallback).  Network: I -> H -> H -> O, GELU(z) = z Phi(z) after both hidden
 * layers, linear output; loss L = sum (y - t)^2 / (2 B O) over a batch of B
 * rows.
 *
 * params: bfloat16, flat, W1 (H x I), b1 (H), W2 (H x H), b2 (H), W3 (O x H),
 * b3 (O), row-major (gnmppi_mlp_param_count elements).  Every matrix product
 * rounds both operands to bfloat16 and accumulates in float32.  X (B x I),
 * Y and T (B x O) are row-major float32.  `work` holds the activations of the
 * last forward pass: gnmppi_mlp_workspace bytes, 256-byte aligned.
 * 1 <= I, H, O <= 4096, 1 <= B <= 1 << 20; otherwise GNMPPI_EINVAL.  Device
 * pointers, owned by the caller; nothing is allocated.                      */
int64_t gnmppi_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out);
size_t gnmppi_mlp_workspace(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch);

/* Y = net(X). */
int gnmppi_mlp_forward(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch,
                       const void *params, const float *X, float *Y, void *work,
                       size_t work_bytes, void *stream);

/* Forward pass, then loss (one float, may be NULL) and its gradient with
 * respect to every parameter, in the parameter layout, float32. */
int gnmppi_mlp_backward(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch,
                        const void *params, const float *X, const float *T, float *loss,
                        float *grad, void *work, size_t work_bytes, void *stream);

/* One Adam step (Kingma and Ba) on `count` parameters: float32 master copy,
 * moments m and v (float32, start at zero), step counted from 1; the bfloat16
 * compute copy `params` is rewritten from the master. */
int gnmppi_mlp_adam(int64_t count, float *master, void *params, const float *grad, float *m,
                    float *v, double lr, double beta1, double beta2, double eps, int32_t step,
                    void *stream);

/* ---- misc ----------------------------------------------------------------- */
const char *gnmppi_status_string(int32_t status);
int32_t gnmppi_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GNMPPI_H */
