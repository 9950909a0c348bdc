"""Helpers for the GPU parity tests: identical dtype-rounded inputs for the
HIP path and the oracle, and the tolerance rule.

Tolerance (the stated bar, read normwise per output array): relative error
||got - ref|| / ||ref|| <= 1e-4 for float32 and <= 1e-10 for float64, plus an
element-wise bound |got - ref| <= tol * max|ref|.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest
import torch

TOL = {"f32": 1e-4, "f64": 1e-10}
NP = {"f32": np.float32, "f64": np.float64}
TORCH = {"f32": torch.float32, "f64": torch.float64}


def device():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X (torch.cuda.is_available() is False)")
    return torch.device("cuda")


def rnd(a, dtype):
    """Round to the working precision and return float64 values."""
    return np.asarray(np.asarray(a, dtype=np.float64).astype(NP[dtype]), dtype=np.float64)


def round_problem(prob, dtype):
    """The problem exactly as the device sees it (every scalar and vector
    rounded to the working precision)."""
    r = lambda v: float(NP[dtype](v))  # noqa: E731
    return dataclasses.replace(prob, dt=r(prob.dt), k_lin=r(prob.k_lin), k_cub=r(prob.k_cub),
                               mass=float(1.0 / NP[dtype](1.0 / prob.mass)) if dtype == "f32" else prob.mass,
                               q=rnd(prob.q, dtype), r=rnd(prob.r, dtype), x_ref=rnd(prob.x_ref, dtype))


def to_dev(a, dtype, dev=None):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(
        device=dev or device(), dtype=TORCH[dtype]).contiguous()


def padded(a, dtype, ld=None, dev=None):
    """Matrix on the device with leading dimension ``ld`` (>= columns)."""
    a = np.asarray(a, dtype=np.float64)
    rows, cols = a.shape
    ld = ld or ((cols + 63) // 64 * 64)
    t = torch.full((rows, ld), float("nan"), dtype=TORCH[dtype], device=dev or device())
    t[:, :cols] = to_dev(a, dtype, dev)
    return t[:, :cols]


def host(t):
    return t.detach().double().cpu().numpy()


def rel_err(got, ref):
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def assert_parity(got, ref, dtype, what="", tol=None):
    tol = TOL[dtype] if tol is None else tol
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got) == np.isfinite(ref)), what
    f = np.isfinite(ref)
    e = rel_err(got[f], ref[f])
    assert e <= tol, f"{what}: normwise relative error {e:.3e} > {tol:.1e}"
    scale = np.abs(ref[f]).max() if f.any() else 1.0
    worst = np.abs(got[f] - ref[f]).max() if f.any() else 0.0
    assert worst <= tol * max(scale, 1e-300), f"{what}: max abs error {worst:.3e} > {tol:.1e} * {scale:.3e}"
    return e
