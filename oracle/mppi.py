"""Deterministic MPPI step, Eqs. (5)-(8) (Sec. 3).  Test infrastructure only.

The empirical step (Eq. (7)) is sum_m W_m w_m / sum_m w_m with
w_m = exp(-C(U_k + W_m) / lambda_k) (Eq. (8)).  Readings: the sum runs over
the M perturbed samples only (the nominal is not a sample); the common factor
exp(min C / lambda) is removed before exponentiating, which leaves the ratio
unchanged and avoids underflow; a sample whose cost is NaN or infinite gets
weight zero, and if no sample has a finite cost the step is undefined.
"""
from __future__ import annotations

import numpy as np


class NoFiniteCost(ValueError):
    pass


def weights(C, temperature: float):
    """Normalised weights w_m / sum w (Eq. (8) divided by the Eq. (7)
    denominator)."""
    C = np.asarray(C, dtype=np.float64)
    finite = np.isfinite(C)
    if not finite.any():
        raise NoFiniteCost("no sample has a finite cost")
    cmin = C[finite].min()
    w = np.zeros_like(C)
    w[finite] = np.exp(-(C[finite] - cmin) / temperature)
    return w / w.sum()


def step(W, C, temperature: float):
    """Delta U_MPPI of Eq. (7); W has shape (n, M) with one sample per column."""
    return np.asarray(W, dtype=np.float64) @ weights(C, temperature)


def update(U, W, C, temperature: float):
    """U_{k+1} = U_k + Delta U_MPPI(U_k) (Sec. 3)."""
    return np.asarray(U, dtype=np.float64) + step(W, C, temperature)
