"""Generalized Gauss-Newton step and parallel line search, Eqs. (13)-(15)
(Sec. 4.2-4.3).  Test infrastructure only.

With Phi = 1/2 ||R||^2 the gradient is J^T R and the GGN Hessian is J^T J,
so Eq. (13) reads  Delta = -(J^T J + lambda I)^{-1} J^T r0  with r0 = R(U_k)
(lambda = 0 is the paper's step; lambda > 0 is an optional regulariser).
"""
from __future__ import annotations

import numpy as np


class NotPositiveDefinite(ValueError):
    pass


def direction(J, r0, lm_lambda: float = 0.0):
    J = np.asarray(J, dtype=np.float64)
    r0 = np.asarray(r0, dtype=np.float64)
    H = J.T @ J + lm_lambda * np.eye(J.shape[1])
    g = J.T @ r0
    try:
        L = np.linalg.cholesky(H)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    y = np.linalg.solve(L, g)
    return -np.linalg.solve(L.T, y)


def step_lengths(gamma: float, count: int):
    """The candidate set A = {gamma^j, j = 0..count-1} of Eq. (15)."""
    return gamma ** np.arange(count, dtype=np.float64)


def line_search(costfun, U, delta, alphas):
    """alpha* = argmin_{alpha in A} C(U + alpha Delta) (Eq. (15)); ties go to
    the first (largest) candidate.  ``costfun`` maps an (n, L) batch of
    control sequences to L costs.  Returns (U_new, alpha*, j*, costs)."""
    U = np.asarray(U, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    alphas = np.asarray(alphas, dtype=np.float64)
    costs = np.asarray(costfun(U[:, None] + delta[:, None] * alphas[None, :]), dtype=np.float64)
    j = int(np.argmin(np.where(np.isfinite(costs), costs, np.inf)))
    return U + alphas[j] * delta, alphas[j], j, costs
