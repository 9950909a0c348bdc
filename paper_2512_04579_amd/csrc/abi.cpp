// C ABI of libgnmppi: argument validation and dispatch to the kernel
// launchers.  Nothing here allocates, synchronises or touches device memory;
// invalid arguments are rejected before any work is enqueued.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gnmppi.h"
#include "launch.hpp"

namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int status_of(hipError_t e) { return e == hipSuccess ? GNMPPI_OK : GNMPPI_EHIP; }

bool dtype_ok(int32_t dtype) { return dtype == GNMPPI_F32 || dtype == GNMPPI_F64; }

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// Model-specific shape rules (see the model descriptions in gnmppi.h).
bool problem_ok(const gnmppi_problem* p) {
  if (p == nullptr || !dtype_ok(p->dtype)) return false;
  if (p->N < 1 || p->nx < 1 || p->nu < 1) return false;
  if (p->q == nullptr || p->r == nullptr || p->x_ref == nullptr) return false;
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return false;
  if (p->model == GNMPPI_MODEL_DOUBLE_INTEGRATOR) {
    return p->nu >= 1 && p->nu <= 4 && p->nx == 2 * p->nu;
  }
  if (p->model == GNMPPI_MODEL_CHAIN) {
    return p->n_masses >= 1 && p->n_masses <= 16 && p->nx == 4 * p->n_masses && p->nu == 2 &&
           p->mass > 0.0 && std::isfinite(p->k_lin) && std::isfinite(p->k_cub);
  }
  return false;
}

// Products below stay in 64-bit; reject horizons whose residual count
// overflows a 32-bit row index.
bool sizes_fit(const gnmppi_problem* p) {
  const int64_t m = static_cast<int64_t>(p->N) * (p->nx + p->nu);
  return m < (int64_t{1} << 30);
}

}  // namespace

extern "C" {

int gnmppi_sample(int32_t dtype, int32_t n, int32_t K, double sigma, uint64_t seed,
                  uint64_t stream_id, int32_t antithetic, void* W, int64_t ldw, void* stream) {
  if (!dtype_ok(dtype) || n < 1 || K < 1 || W == nullptr || ldw < K) return GNMPPI_EINVAL;
  if (antithetic && (K % 2) != 0) return GNMPPI_EINVAL;
  if (!std::isfinite(sigma) || n > 65535 * 2) return GNMPPI_EINVAL;
  return status_of(gnm::launch_sample(dtype, n, K, sigma, seed, stream_id, antithetic != 0, W, ldw,
                                      as_stream(stream)));
}

int gnmppi_sigma_points(int32_t dtype, int32_t n, double sigma, void* W, int64_t ldw,
                        void* stream) {
  if (!dtype_ok(dtype) || n < 1 || n > 65535 || W == nullptr || ldw < 2 * static_cast<int64_t>(n))
    return GNMPPI_EINVAL;
  if (!std::isfinite(sigma)) return GNMPPI_EINVAL;
  return status_of(gnm::launch_sigma_points(dtype, n, sigma, W, ldw, as_stream(stream)));
}

int gnmppi_rollout(const gnmppi_problem* p, const void* x0, const void* U, const void* W,
                   int64_t ldw, int32_t K, void* R, int64_t ldr, void* C, void* r0, void* c0,
                   void* stream) {
  if (!problem_ok(p) || !sizes_fit(p) || x0 == nullptr || U == nullptr) return GNMPPI_EINVAL;
  if (K < 0 || (K == 0 && c0 == nullptr)) return GNMPPI_EINVAL;
  if (K > 0) {
    if (C == nullptr && R == nullptr) return GNMPPI_EINVAL;  // nothing wanted of the K columns
    if (W != nullptr && ldw < K) return GNMPPI_EINVAL;
    if (R != nullptr && ldr < K) return GNMPPI_EINVAL;
  }
  if (r0 != nullptr && c0 == nullptr) return GNMPPI_EINVAL;
  if (static_cast<int64_t>(K) * 16 >= (int64_t{1} << 31)) return GNMPPI_EINVAL;
  return status_of(gnm::launch_rollout(*p, x0, U, W, ldw, K, K > 0 ? R : nullptr, ldr, C, r0, c0,
                                       as_stream(stream)));
}

int gnmppi_sample_rollout(const gnmppi_problem* p, const void* x0, const void* U, double sigma,
                          uint64_t seed, uint64_t stream_id, int32_t antithetic, void* W,
                          int64_t ldw, int32_t K, void* R, int64_t ldr, void* C, void* r0,
                          void* c0, void* stream) {
  if (!problem_ok(p) || !sizes_fit(p) || x0 == nullptr || U == nullptr || W == nullptr)
    return GNMPPI_EINVAL;
  if (K < 1 || ldw < K || (antithetic && (K % 2) != 0) || !std::isfinite(sigma))
    return GNMPPI_EINVAL;
  if (static_cast<int64_t>(p->N) * p->nu > 65535 * 2) return GNMPPI_EINVAL;
  if (C == nullptr && R == nullptr) return GNMPPI_EINVAL;
  if (R != nullptr && ldr < K) return GNMPPI_EINVAL;
  if (r0 != nullptr && c0 == nullptr) return GNMPPI_EINVAL;
  if (static_cast<int64_t>(K) * 16 >= (int64_t{1} << 31)) return GNMPPI_EINVAL;
  return status_of(gnm::launch_sample_rollout(*p, x0, U, sigma, seed, stream_id, antithetic != 0,
                                              W, ldw, K, R, ldr, C, r0, c0, as_stream(stream)));
}

int gnmppi_mppi_update(int32_t dtype, int32_t n, int32_t K, const void* C, const void* W,
                       int64_t ldw, double temperature, void* U, void* weights, int32_t* status,
                       void* stream) {
  if (!dtype_ok(dtype) || n < 1 || K < 1 || C == nullptr || W == nullptr || U == nullptr)
    return GNMPPI_EINVAL;
  if (ldw < K || !(temperature > 0.0) || !std::isfinite(temperature)) return GNMPPI_EINVAL;
  const int32_t kmax = dtype == GNMPPI_F32 ? 16384 : 8192;  // weights live in 64 KB of LDS
  if (K > kmax) return GNMPPI_EINVAL;
  return status_of(gnm::launch_mppi_update(dtype, n, K, C, W, ldw, temperature, U, weights, status,
                                           as_stream(stream)));
}

size_t gnmppi_jacobian_workspace(int32_t dtype, int32_t m, int32_t n, int32_t K) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || K < 1) return 0;
  return gnm::jacobian_plan(dtype, m, n, K, GNMPPI_JAC_LS).total;
}

int gnmppi_reconstruct_jacobian(int32_t dtype, int32_t m, int32_t n, int32_t K, const void* R,
                                int64_t ldr, const void* r0, const void* W, int64_t ldw,
                                int32_t method, double sigma2, void* J, int64_t ldj, void* work,
                                size_t work_bytes, int32_t* status, void* stream) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || n > 192 || K < 1) return GNMPPI_EINVAL;
  if (R == nullptr || r0 == nullptr || W == nullptr || J == nullptr || work == nullptr)
    return GNMPPI_EINVAL;
  if (ldr < K || ldw < K || ldj < n) return GNMPPI_EINVAL;
  const int32_t base = method & 0xff, flags = method & ~0xff;
  if (base != GNMPPI_JAC_LS && base != GNMPPI_JAC_MC) return GNMPPI_EINVAL;
  if (flags & ~(GNMPPI_JAC_GRAM_READY | GNMPPI_JAC_BF16 | GNMPPI_JAC_BF16X3 | GNMPPI_JAC_S_ONLY |
                GNMPPI_JAC_APPLY_ONLY))
    return GNMPPI_EINVAL;
  if ((flags & GNMPPI_JAC_GRAM_READY) && base != GNMPPI_JAC_LS) return GNMPPI_EINVAL;
  if ((flags & (GNMPPI_JAC_S_ONLY | GNMPPI_JAC_APPLY_ONLY)) && !(flags & GNMPPI_JAC_GRAM_READY))
    return GNMPPI_EINVAL;
  if ((flags & GNMPPI_JAC_S_ONLY) && (flags & GNMPPI_JAC_APPLY_ONLY)) return GNMPPI_EINVAL;
  if ((flags & GNMPPI_JAC_BF16) && (flags & GNMPPI_JAC_BF16X3)) return GNMPPI_EINVAL;
  if ((flags & (GNMPPI_JAC_BF16 | GNMPPI_JAC_BF16X3)) && dtype != GNMPPI_F32) return GNMPPI_EINVAL;
  if (base == GNMPPI_JAC_MC && (!(sigma2 > 0.0) || !std::isfinite(sigma2))) return GNMPPI_EINVAL;
  if (!aligned256(work)) return GNMPPI_EINVAL;
  if (work_bytes < gnm::jacobian_plan(dtype, m, n, K, method).total) return GNMPPI_ENOSPACE;
  if (static_cast<int64_t>(m + n) * 192 >= (int64_t{1} << 31)) return GNMPPI_EINVAL;
  return status_of(gnm::launch_jacobian(dtype, m, n, K, R, ldr, r0, W, ldw, method, sigma2, J, ldj,
                                        work, status, as_stream(stream)));
}

int gnmppi_perturbation_gram(int32_t dtype, int32_t m, int32_t n, int32_t K, const void* W,
                             int64_t ldw, void* work, size_t work_bytes, int32_t* status,
                             void* stream) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || n > 192 || K < 1) return GNMPPI_EINVAL;
  if (W == nullptr || work == nullptr || ldw < K || !aligned256(work)) return GNMPPI_EINVAL;
  if (work_bytes < gnm::jacobian_plan(dtype, m, n, K, GNMPPI_JAC_LS).total) return GNMPPI_ENOSPACE;
  return status_of(gnm::launch_gram(dtype, m, n, K, W, ldw, work, status, as_stream(stream)));
}

size_t gnmppi_ggn_workspace(int32_t dtype, int32_t m, int32_t n) {
  if (!dtype_ok(dtype) || m < 1 || n < 1) return 0;
  return gnm::ggn_plan(dtype, m, n).total;
}

int gnmppi_ggn_step(int32_t dtype, int32_t m, int32_t n, const void* J, int64_t ldj,
                    const void* r0, int64_t inc_r0, double lm_lambda, void* dU, void* work,
                    size_t work_bytes, int32_t* status, void* stream) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || n > 192) return GNMPPI_EINVAL;
  if (J == nullptr || r0 == nullptr || dU == nullptr || work == nullptr) return GNMPPI_EINVAL;
  if (ldj < n || inc_r0 < 1 || !(lm_lambda >= 0.0) || !std::isfinite(lm_lambda))
    return GNMPPI_EINVAL;
  if (!aligned256(work)) return GNMPPI_EINVAL;
  if (work_bytes < gnm::ggn_plan(dtype, m, n).total) return GNMPPI_ENOSPACE;
  return status_of(gnm::launch_ggn(dtype, m, n, J, ldj, r0, inc_r0, lm_lambda, dU, work, status,
                                   as_stream(stream)));
}

size_t gnmppi_ggn_direction_workspace(int32_t dtype, int32_t m, int32_t n, int32_t K) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || K < 1) return 0;
  return gnm::ggn_direction_bytes(dtype, m, n, K);
}

int gnmppi_ggn_direction(int32_t dtype, int32_t m, int32_t n, int32_t K, const void* R,
                         int64_t ldr, const void* r0, const void* W, int64_t ldw, int32_t method,
                         double sigma2, double lm_lambda, void* dU, void* work, size_t work_bytes,
                         int32_t* status, void* stream) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || n > 192 || K < 1) return GNMPPI_EINVAL;
  if (R == nullptr || r0 == nullptr || W == nullptr || dU == nullptr || work == nullptr)
    return GNMPPI_EINVAL;
  if (ldr < K || ldw < K) return GNMPPI_EINVAL;
  const int32_t base = method & 0xff, flags = method & ~0xff;
  if (flags & ~(GNMPPI_JAC_GRAM_READY | GNMPPI_JAC_BF16 | GNMPPI_JAC_BF16X3 | GNMPPI_JAC_S_ONLY |
                GNMPPI_JAC_APPLY_ONLY))
    return GNMPPI_EINVAL;
  // MC has no G (and nothing to split around it)
  if (base == GNMPPI_JAC_MC) {
    if (flags & (GNMPPI_JAC_GRAM_READY | GNMPPI_JAC_S_ONLY | GNMPPI_JAC_APPLY_ONLY))
      return GNMPPI_EINVAL;
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return GNMPPI_EINVAL;
  } else if (base != GNMPPI_JAC_LS) {
    return GNMPPI_EINVAL;
  }
  if ((flags & GNMPPI_JAC_S_ONLY) && (flags & GNMPPI_JAC_APPLY_ONLY)) return GNMPPI_EINVAL;
  if ((flags & GNMPPI_JAC_BF16) && (flags & GNMPPI_JAC_BF16X3)) return GNMPPI_EINVAL;
  if ((flags & (GNMPPI_JAC_BF16 | GNMPPI_JAC_BF16X3)) && dtype != GNMPPI_F32) return GNMPPI_EINVAL;
  if (!(lm_lambda >= 0.0) || !std::isfinite(lm_lambda)) return GNMPPI_EINVAL;
  if (!aligned256(work)) return GNMPPI_EINVAL;
  if (work_bytes < gnm::ggn_direction_bytes(dtype, m, n, K)) return GNMPPI_ENOSPACE;
  if (static_cast<int64_t>(m + n) * 192 >= (int64_t{1} << 31)) return GNMPPI_EINVAL;
  return status_of(gnm::launch_ggn_direction(dtype, m, n, K, R, ldr, r0, W, ldw, method, sigma2,
                                             lm_lambda, dU, work, status, as_stream(stream)));
}

int gnmppi_ggn_step_noalloc(int32_t dtype, int32_t m, int32_t n, const void* J, int64_t ldj,
                            const void* r0, int64_t inc_r0, double lm_lambda, void* dU,
                            int32_t* status, void* stream) {
  if (!dtype_ok(dtype) || m < 1 || n < 1 || n > 192) return GNMPPI_EINVAL;
  if (J == nullptr || r0 == nullptr || dU == nullptr) return GNMPPI_EINVAL;
  if (ldj < n || inc_r0 < 1 || !(lm_lambda >= 0.0) || !std::isfinite(lm_lambda))
    return GNMPPI_EINVAL;
  if (gnm::ggn_plan(dtype, m, n).total > gnm::ggn_noalloc_capacity()) return GNMPPI_ENOSPACE;
  return status_of(gnm::launch_ggn_noalloc(dtype, m, n, J, ldj, r0, inc_r0, lm_lambda, dU, status,
                                           as_stream(stream)));
}

int gnmppi_line_search(const gnmppi_problem* p, const void* x0, void* U, const void* dU,
                       const void* alpha, int32_t L, void* C, double* info, int32_t* status,
                       void* stream) {
  if (!problem_ok(p) || !sizes_fit(p) || x0 == nullptr || U == nullptr || dU == nullptr ||
      alpha == nullptr)
    return GNMPPI_EINVAL;
  if (L < 1 || L > 64) return GNMPPI_EINVAL;
  return status_of(
      gnm::launch_line_search(*p, x0, U, dU, alpha, L, C, info, status, as_stream(stream)));
}

int gnmppi_line_search_nominal(const gnmppi_problem* p, const void* x0, void* U, const void* dU,
                               const void* alpha, int32_t L, void* C, double* info,
                               int32_t* status, void* Rc, void* r0, void* c0, void* stream) {
  if (!problem_ok(p) || !sizes_fit(p) || x0 == nullptr || U == nullptr || dU == nullptr ||
      alpha == nullptr || Rc == nullptr || r0 == nullptr || c0 == nullptr)
    return GNMPPI_EINVAL;
  if (L < 1 || L > 64) return GNMPPI_EINVAL;
  return status_of(gnm::launch_line_search(*p, x0, U, dU, alpha, L, C, info, status,
                                           as_stream(stream), Rc, r0, c0));
}

int64_t gnmppi_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out) {
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || n_in > 4096 || n_hidden > 4096 || n_out > 4096)
    return 0;
  return gnm::mlp_param_count(n_in, n_hidden, n_out);
}

size_t gnmppi_mlp_workspace(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch) {
  if (gnmppi_mlp_param_count(n_in, n_hidden, n_out) == 0 || batch < 1 || batch > (1 << 20)) return 0;
  return gnm::mlp_workspace_bytes(n_hidden, n_out, batch);
}

int gnmppi_mlp_forward(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch,
                       const void* params, const float* X, float* Y, void* work, size_t work_bytes,
                       void* stream) {
  const size_t need = gnmppi_mlp_workspace(n_in, n_hidden, n_out, batch);
  if (need == 0 || params == nullptr || X == nullptr || Y == nullptr || work == nullptr ||
      !aligned256(work))
    return GNMPPI_EINVAL;
  if (work_bytes < need) return GNMPPI_ENOSPACE;
  return status_of(gnm::launch_mlp_forward(n_in, n_hidden, n_out, batch, params, X, Y, work,
                                           as_stream(stream)));
}

int gnmppi_mlp_backward(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch,
                        const void* params, const float* X, const float* T, float* loss,
                        float* grad, void* work, size_t work_bytes, void* stream) {
  const size_t need = gnmppi_mlp_workspace(n_in, n_hidden, n_out, batch);
  if (need == 0 || params == nullptr || X == nullptr || T == nullptr || grad == nullptr ||
      work == nullptr || !aligned256(work))
    return GNMPPI_EINVAL;
  if (work_bytes < need) return GNMPPI_ENOSPACE;
  return status_of(gnm::launch_mlp_backward(n_in, n_hidden, n_out, batch, params, X, T, loss, grad,
                                            work, as_stream(stream)));
}

int gnmppi_mlp_adam(int64_t count, float* master, void* params, const float* grad, float* m,
                    float* v, double lr, double beta1, double beta2, double eps, int32_t step,
                    void* stream) {
  if (count < 1 || master == nullptr || params == nullptr || grad == nullptr || m == nullptr ||
      v == nullptr || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0) || count > (int64_t{1} << 40))
    return GNMPPI_EINVAL;
  return status_of(gnm::launch_mlp_adam(count, master, params, grad, m, v, lr, beta1, beta2, eps,
                                        step, as_stream(stream)));
}

const char* gnmppi_status_string(int32_t status) {
  switch (status) {
    case GNMPPI_OK: return "ok";
    case GNMPPI_EINVAL: return "invalid argument";
    case GNMPPI_EHIP: return "HIP runtime error";
    case GNMPPI_ENOTPD: return "normal matrix not positive definite";
    case GNMPPI_ERANK: return "perturbations do not span the decision space";
    case GNMPPI_ENONFINITE: return "no finite cost";
    case GNMPPI_ENOSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

int32_t gnmppi_abi_version(void) { return 4; }

}  // extern "C"
