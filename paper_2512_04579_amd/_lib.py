"""ctypes binding of libgnmppi.so (declared in include/gnmppi.h).

Argument marshalling only: every function forwards device pointers, sizes
and the current torch stream to the C entry point of the same name, and
raises ``GnmppiError`` on a non-zero return.  There is no fallback: if the
shared library is missing the import of the first call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgnmppi.so")

F32, F64 = 0, 1
MODEL_DOUBLE_INTEGRATOR, MODEL_CHAIN = 1, 2
JAC_LS, JAC_MC = 0, 1
JAC_GRAM_READY = 0x100
JAC_BF16, JAC_BF16X3 = 0x200, 0x400
JAC_S_ONLY, JAC_APPLY_ONLY = 0x800, 0x1000
OK, EINVAL, EHIP, ENOTPD, ERANK, ENONFINITE, ENOSPACE = 0, -1, -2, -3, -4, -5, -6


class GnmppiError(RuntimeError):
    def __init__(self, func: str, code: int, message: str):
        super().__init__(f"{func} returned {code}: {message}")
        self.code = code


class GnmppiProblem(ctypes.Structure):
    """Mirror of ``gnmppi_problem``."""

    _fields_ = [
        ("model", c_int32), ("dtype", c_int32), ("nx", c_int32), ("nu", c_int32),
        ("N", c_int32), ("n_masses", c_int32),
        ("dt", c_double), ("k_lin", c_double), ("k_cub", c_double), ("mass", c_double),
        ("q", c_void_p), ("r", c_void_p), ("x_ref", c_void_p),
    ]


class GnmppiBatchInstance(ctypes.Structure):
    """Mirror of ``gnmppi_batch_instance``."""

    _fields_ = [
        ("n_masses", c_int32), ("N", c_int32), ("K", c_int32), ("reserved", c_int32),
        ("x0", c_void_p), ("q", c_void_p), ("r", c_void_p), ("x_ref", c_void_p),
        ("U", c_void_p), ("status", c_void_p), ("info", c_void_p),
    ]


class GnmppiBatchSettings(ctypes.Structure):
    _fields_ = [("seed", c_uint64), ("gamma", c_double), ("n_alpha", c_int32),
                ("reserved", c_int32), ("lm_lambda", c_double)]


class GnmppiBatchTuning(ctypes.Structure):
    _fields_ = [("rollout_blocks_per_cu", c_int32), ("contract_blocks_per_cu", c_int32),
                ("contract_ksplit", c_int32), ("small_blocks_per_cu", c_int32),
                ("rollout_mode", c_int32)]


PROBLEM_P = ctypes.POINTER(GnmppiProblem)
BATCH_P = ctypes.POINTER(GnmppiBatchInstance)
BSET_P = ctypes.POINTER(GnmppiBatchSettings)
BTUNE_P = ctypes.POINTER(GnmppiBatchTuning)
I32_P = ctypes.POINTER(c_int32)
F64_P = ctypes.POINTER(c_double)

SIGNATURES = {
    "gnmppi_sample": (c_int32, [c_int32, c_int32, c_int32, c_double, c_uint64, c_uint64, c_int32,
                                c_void_p, c_int64, c_void_p]),
    "gnmppi_sigma_points": (c_int32, [c_int32, c_int32, c_double, c_void_p, c_int64, c_void_p]),
    "gnmppi_rollout": (c_int32, [PROBLEM_P, c_void_p, c_void_p, c_void_p, c_int64, c_int32,
                                 c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gnmppi_sample_rollout": (c_int32, [PROBLEM_P, c_void_p, c_void_p, c_double, c_uint64, c_uint64,
                                        c_int32, c_void_p, c_int64, c_int32, c_void_p, c_int64,
                                        c_void_p, c_void_p, c_void_p, c_void_p]),
    "gnmppi_mppi_update": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int64,
                                     c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gnmppi_jacobian_workspace": (c_size_t, [c_int32, c_int32, c_int32, c_int32]),
    "gnmppi_reconstruct_jacobian": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p,
                                              c_int64, c_void_p, c_void_p, c_int64, c_int32,
                                              c_double, c_void_p, c_int64, c_void_p, c_size_t,
                                              c_void_p, c_void_p]),
    "gnmppi_perturbation_gram": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_int64,
                                           c_void_p, c_size_t, c_void_p, c_void_p]),
    "gnmppi_ggn_workspace": (c_size_t, [c_int32, c_int32, c_int32]),
    "gnmppi_ggn_step": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                                  c_double, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "gnmppi_ggn_direction_workspace": (c_size_t, [c_int32, c_int32, c_int32, c_int32]),
    "gnmppi_ggn_direction": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_int64,
                                       c_void_p, c_void_p, c_int64, c_int32, c_double, c_double,
                                       c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "gnmppi_ggn_step_noalloc": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int64, c_void_p,
                                          c_int64, c_double, c_void_p, c_void_p, c_void_p]),
    "gnmppi_line_search": (c_int32, [PROBLEM_P, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                     c_void_p, c_void_p, c_void_p, c_void_p]),
    "gnmppi_line_search_nominal": (c_int32, [PROBLEM_P, c_void_p, c_void_p, c_void_p, c_void_p,
                                             c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                             c_void_p, c_void_p, c_void_p]),
    "gnmppi_batch_workspace": (c_size_t, [PROBLEM_P, c_int32, BATCH_P, BSET_P, BTUNE_P]),
    "gnmppi_batch_prepare": (c_int32, [PROBLEM_P, c_int32, BATCH_P, BSET_P, BTUNE_P, c_void_p, c_size_t]),
    "gnmppi_batch_iteration": (c_int32, [PROBLEM_P, c_int32, BATCH_P, BSET_P, BTUNE_P, c_void_p,
                                         c_size_t, c_int32, c_double, c_void_p]),
    "gnmppi_mlp_param_count": (c_int64, [c_int32, c_int32, c_int32]),
    "gnmppi_mlp_workspace": (c_size_t, [c_int32, c_int32, c_int32, c_int32]),
    "gnmppi_mlp_forward": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]),
    "gnmppi_mlp_backward": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gnmppi_mlp_adam": (c_int32, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                  c_double, c_double, c_double, c_int32, c_void_p]),
    "gnmppi_status_string": (ctypes.c_char_p, [c_int32]),
    "gnmppi_abi_version": (c_int32, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (once) and declare every signature."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the HIP runtime that torch brings must be the one the
    # library binds to, or the process holds two runtimes and the library's
    # calls do not know torch's allocations and streams
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it first (python -m paper_2512_04579_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().gnmppi_status_string(int(code)).decode()


def _check(name: str, code: int):
    if code != OK:
        raise GnmppiError(name, code, status_string(code))


# ---------------------------------------------------------------------------
# tensor marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _ld(t, default: int = 0) -> int:
    if t is None:
        return default
    if t.dim() == 1:
        return t.numel()
    if t.stride(1) != 1:
        raise ValueError("matrices must be row-major with unit column stride")
    return t.stride(0)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# entry points (same names and argument order as the C ABI)
# ---------------------------------------------------------------------------

def gnmppi_sample(W, sigma: float, seed: int, stream_id: int, antithetic: bool = True,
                  K: int | None = None, stream=None):
    n = W.shape[0]
    K = W.shape[1] if K is None else K
    _check("gnmppi_sample", load().gnmppi_sample(
        _dtype_code(W), n, K, float(sigma), int(seed) & (2 ** 64 - 1),
        int(stream_id) & (2 ** 64 - 1), int(bool(antithetic)), _ptr(W), _ld(W), _stream(stream)))


def gnmppi_sigma_points(W, sigma: float, stream=None):
    n = W.shape[0]
    _check("gnmppi_sigma_points", load().gnmppi_sigma_points(
        _dtype_code(W), n, float(sigma), _ptr(W), _ld(W), _stream(stream)))


def gnmppi_rollout(problem, x0, U, W, K: int, R=None, C=None, r0=None, c0=None, stream=None):
    """``problem`` is a ``DeviceProblem`` (see ``problem.py``)."""
    _check("gnmppi_rollout", load().gnmppi_rollout(
        ctypes.byref(problem.c), _ptr(x0), _ptr(U), _ptr(W), _ld(W), int(K), _ptr(R), _ld(R),
        _ptr(C), _ptr(r0), _ptr(c0), _stream(stream)))


def gnmppi_sample_rollout(problem, x0, U, W, sigma: float, seed: int, stream_id: int, K: int,
                          antithetic: bool = True, R=None, C=None, r0=None, c0=None, stream=None):
    """gnmppi_sample into ``W`` and gnmppi_rollout of U + W in one call."""
    _check("gnmppi_sample_rollout", load().gnmppi_sample_rollout(
        ctypes.byref(problem.c), _ptr(x0), _ptr(U), float(sigma), int(seed) & (2 ** 64 - 1),
        int(stream_id) & (2 ** 64 - 1), 1 if antithetic else 0, _ptr(W), _ld(W), int(K), _ptr(R), _ld(R), _ptr(C), _ptr(r0),
        _ptr(c0), _stream(stream)))


def gnmppi_mppi_update(C, W, temperature: float, U, weights=None, status=None, K: int | None = None,
                       stream=None):
    n = U.numel()
    K = C.numel() if K is None else K
    _check("gnmppi_mppi_update", load().gnmppi_mppi_update(
        _dtype_code(U), n, K, _ptr(C), _ptr(W), _ld(W), float(temperature), _ptr(U),
        _ptr(weights), _ptr(status), _stream(stream)))


def gnmppi_jacobian_workspace(dtype: int, m: int, n: int, K: int) -> int:
    return int(load().gnmppi_jacobian_workspace(dtype, m, n, K))


def gnmppi_reconstruct_jacobian(R, r0, W, J, work, method: int = JAC_LS, sigma2: float = 0.0,
                                status=None, K: int | None = None, stream=None):
    m, n = J.shape
    K = W.shape[1] if K is None else K
    _check("gnmppi_reconstruct_jacobian", load().gnmppi_reconstruct_jacobian(
        _dtype_code(J), m, n, K, _ptr(R), _ld(R), _ptr(r0), _ptr(W), _ld(W), int(method),
        float(sigma2), _ptr(J), _ld(J), _ptr(work), work.numel() * work.element_size(),
        _ptr(status), _stream(stream)))


def gnmppi_perturbation_gram(W, work, m: int, status=None, K: int | None = None, stream=None):
    n = W.shape[0]
    K = W.shape[1] if K is None else K
    _check("gnmppi_perturbation_gram", load().gnmppi_perturbation_gram(
        _dtype_code(W), int(m), n, K, _ptr(W), _ld(W), _ptr(work),
        work.numel() * work.element_size(), _ptr(status), _stream(stream)))


def gnmppi_ggn_workspace(dtype: int, m: int, n: int) -> int:
    return int(load().gnmppi_ggn_workspace(dtype, m, n))


def gnmppi_ggn_step(J, r0, lm_lambda: float, dU, work, status=None, inc_r0: int = 1, stream=None):
    m, n = J.shape
    _check("gnmppi_ggn_step", load().gnmppi_ggn_step(
        _dtype_code(J), m, n, _ptr(J), _ld(J), _ptr(r0), int(inc_r0), float(lm_lambda), _ptr(dU),
        _ptr(work), work.numel() * work.element_size(), _ptr(status), _stream(stream)))


def gnmppi_ggn_direction_workspace(dtype: int, m: int, n: int, K: int) -> int:
    return int(load().gnmppi_ggn_direction_workspace(dtype, m, n, K))


def gnmppi_ggn_direction(R, r0, W, dU, work, method: int, sigma2: float = 0.0,
                         lm_lambda: float = 0.0, status=None, m: int | None = None,
                         K: int | None = None, stream=None):
    m = r0.numel() if m is None else m
    n = dU.numel()
    K = W.shape[1] if K is None else K
    _check("gnmppi_ggn_direction", load().gnmppi_ggn_direction(
        _dtype_code(dU), int(m), n, K, _ptr(R), _ld(R), _ptr(r0), _ptr(W), _ld(W), int(method),
        float(sigma2), float(lm_lambda), _ptr(dU), _ptr(work), work.numel() * work.element_size(),
        _ptr(status), _stream(stream)))


def gnmppi_ggn_step_noalloc(J, r0, lm_lambda: float, dU, status=None, inc_r0: int = 1,
                            stream=None):
    m, n = J.shape
    _check("gnmppi_ggn_step_noalloc", load().gnmppi_ggn_step_noalloc(
        _dtype_code(J), m, n, _ptr(J), _ld(J), _ptr(r0), int(inc_r0), float(lm_lambda), _ptr(dU),
        _ptr(status), _stream(stream)))


def gnmppi_line_search(problem, x0, U, dU, alpha, C=None, info=None, status=None, stream=None):
    _check("gnmppi_line_search", load().gnmppi_line_search(
        ctypes.byref(problem.c), _ptr(x0), _ptr(U), _ptr(dU), _ptr(alpha), alpha.numel(), _ptr(C),
        _ptr(info), _ptr(status), _stream(stream)))


def gnmppi_line_search_nominal(problem, x0, U, dU, alpha, Rc, r0, c0, C=None, info=None,
                               status=None, stream=None):
    """gnmppi_line_search that also writes r0, c0 of the updated controls;
    Rc: scratch of alpha.numel() * r0.numel() entries."""
    _check("gnmppi_line_search_nominal", load().gnmppi_line_search_nominal(
        ctypes.byref(problem.c), _ptr(x0), _ptr(U), _ptr(dU), _ptr(alpha), alpha.numel(), _ptr(C),
        _ptr(info), _ptr(status), _ptr(Rc), _ptr(r0), _ptr(c0), _stream(stream)))


def gnmppi_batch_workspace(shared, count, inst, settings, tuning) -> int:
    return int(load().gnmppi_batch_workspace(ctypes.byref(shared), int(count), inst,
                                             ctypes.byref(settings), ctypes.byref(tuning)))


def gnmppi_batch_prepare(shared, count, inst, settings, tuning, work):
    _check("gnmppi_batch_prepare", load().gnmppi_batch_prepare(
        ctypes.byref(shared), int(count), inst, ctypes.byref(settings), ctypes.byref(tuning),
        _ptr(work), _nbytes(work)))


def gnmppi_batch_iteration(shared, count, inst, settings, tuning, work, it: int, sigma: float,
                           stream=None):
    _check("gnmppi_batch_iteration", load().gnmppi_batch_iteration(
        ctypes.byref(shared), int(count), inst, ctypes.byref(settings), ctypes.byref(tuning),
        _ptr(work), _nbytes(work), int(it), float(sigma), _stream(stream)))


def gnmppi_mlp_param_count(n_in: int, n_hidden: int, n_out: int) -> int:
    return int(load().gnmppi_mlp_param_count(n_in, n_hidden, n_out))


def gnmppi_mlp_workspace(n_in: int, n_hidden: int, n_out: int, batch: int) -> int:
    return int(load().gnmppi_mlp_workspace(n_in, n_hidden, n_out, batch))


def _nbytes(t):
    return t.numel() * t.element_size()


def gnmppi_mlp_forward(dims, params, X, Y, work, stream=None):
    """dims = (n_in, n_hidden, n_out); params bfloat16; X (B, I), Y (B, O) float32."""
    I, H, O = dims
    _check("gnmppi_mlp_forward", load().gnmppi_mlp_forward(
        I, H, O, X.shape[0], _ptr(params), _ptr(X), _ptr(Y), _ptr(work), _nbytes(work), _stream(stream)))


def gnmppi_mlp_backward(dims, params, X, T, loss, grad, work, stream=None):
    I, H, O = dims
    _check("gnmppi_mlp_backward", load().gnmppi_mlp_backward(
        I, H, O, X.shape[0], _ptr(params), _ptr(X), _ptr(T), _ptr(loss), _ptr(grad), _ptr(work),
        _nbytes(work), _stream(stream)))


def gnmppi_mlp_adam(master, params, grad, m, v, lr: float, step: int, beta1: float = 0.9,
                    beta2: float = 0.999, eps: float = 1e-8, stream=None):
    _check("gnmppi_mlp_adam", load().gnmppi_mlp_adam(
        master.numel(), _ptr(master), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), float(lr),
        float(beta1), float(beta2), float(eps), int(step), _stream(stream)))


def gnmppi_abi_version() -> int:
    return int(load().gnmppi_abi_version())
