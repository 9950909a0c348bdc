"""Jacobian reconstruction by Gaussian smoothing, Eq. (10) (Sec. 4.1), and
finite differences (Method A, Sec. 5).  Test infrastructure only.

Inputs follow the hot path's layout: ``R`` is (m, K+1) with column 0 the
nominal residual R(U) and column s+1 the residual at U + W[:, s]; ``W`` is
(n, K).

Two estimators of the smoothed Jacobian dR^/dU = E[R(U+W) W^T] Sigma^{-1}:

* ``mc``: the Monte-Carlo mean of Eq. (10) taken literally, with the nominal
  residual subtracted (which has zero mean against W, so it leaves the
  expectation unchanged):  J = (1/K) sum_s (R_s - R_0) W_s^T Sigma^{-1}.
* ``ls`` (default reading): Sigma replaced by the empirical second moment
  (1/K) W W^T, i.e. the least-squares fit of the residual differences to the
  perturbations,  J = (dR W^T)(W W^T)^{-1}.  It is exact for affine R and, with
  antithetic pairs, for quadratic R.
"""
from __future__ import annotations

import numpy as np


class RankDeficient(ValueError):
    pass


def differences(R):
    R = np.asarray(R, dtype=np.float64)
    return R[:, 1:] - R[:, :1]


def ls(R, W):
    """Least-squares reconstruction J = argmin_J ||dR - J W||_F."""
    W = np.asarray(W, dtype=np.float64)
    dR = differences(R)
    S = dR @ W.T
    G = W @ W.T
    if np.linalg.matrix_rank(W) < W.shape[0]:
        raise RankDeficient("perturbations do not span R^n")
    # J G = S with G symmetric positive definite
    return np.linalg.solve(G, S.T).T


def mc(R, W, sigma2):
    """Monte-Carlo form of Eq. (10) with diagonal Sigma = diag(sigma2)."""
    W = np.asarray(W, dtype=np.float64)
    K = W.shape[1]
    dR = differences(R)
    sigma2 = np.broadcast_to(np.asarray(sigma2, dtype=np.float64), (W.shape[0],))
    return (dR @ W.T) / K / sigma2[None, :]


def central_fd(resfun, U, h: float):
    """J[:, i] = (R(U + h e_i) - R(U - h e_i)) / (2 h), evaluated as one batch."""
    U = np.asarray(U, dtype=np.float64)
    n = U.size
    E = h * np.eye(n)
    Rp = resfun(U[:, None] + E)
    Rm = resfun(U[:, None] - E)
    return (Rp - Rm) / (2.0 * h)
