"""Deterministic Dirac-mixture perturbations for Method E (Sec. 5).
Test infrastructure only.

The paper names the sigma-point construction of the unscented Kalman filter
without fixing its scaling.  Reading: the 2n points +/- sqrt(n) sigma_i e_i
with equal weights 1/(2n).  Their mean is zero and their second moment is
exactly Sigma = diag(sigma^2), so the Monte-Carlo and least-squares forms of
Eq. (10) coincide on this set.
"""
from __future__ import annotations

import numpy as np


def symmetric_set(n: int, sigma):
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (n,))
    D = np.sqrt(n) * np.diag(sigma)
    return np.concatenate([D, -D], axis=1)
