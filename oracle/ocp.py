"""Single-shooting rollouts, residual R and cost C = Phi(R) (Sec. 2,
Eqs. (1), (2) and (4)).  Test infrastructure only.

Residual convention (the reading used throughout): Phi(R) = 1/2 ||R||^2 as in
Problem I, and for each step k = 0..N-1 the residual holds

    sqrt(2 q) * (x_{k+1} - x_ref)   (nx rows)   then
    sqrt(2 r) * u_k                 (nu rows),

so that 1/2 ||R||^2 = sum_k (x_{k+1}-x_ref)^T Q (x_{k+1}-x_ref) + u_k^T R u_k,
i.e. Eq. (2) with stage cost on x_1..x_{N-1}, terminal weight Q_N = Q and the
constant x_0 term dropped (its rows would have zero Jacobian).
m = N (nx + nu) rows, n = N nu decision variables, U stacked time-major.
"""
from __future__ import annotations

import numpy as np

from . import dynamics


def simulate(problem, x0, U):
    """X = F(x0, U) of Eq. (1): states x_0..x_N, shape (N+1, nx) for a single
    U of shape (n,), or (N+1, K, nx) for a batch U of shape (n, K)."""
    U = np.asarray(U, dtype=np.float64)
    N, nu = problem.N, problem.nu
    batch = U.ndim == 2
    if batch:
        Ut = U.reshape(N, nu, -1).transpose(0, 2, 1)  # (N, K, nu)
        x = np.broadcast_to(np.asarray(x0, dtype=np.float64), (U.shape[1], problem.nx)).copy()
    else:
        Ut = U.reshape(N, nu)
        x = np.asarray(x0, dtype=np.float64).copy()
    X = [x]
    for k in range(N):
        x = dynamics.step(problem, x, Ut[k])
        X.append(x)
    return np.stack(X)


def residual_from_states(problem, X, U):
    """R(U) from a simulated trajectory (single or batched)."""
    U = np.asarray(U, dtype=np.float64)
    N, nx, nu = problem.N, problem.nx, problem.nu
    sq = np.sqrt(2.0 * np.asarray(problem.q, dtype=np.float64))
    sr = np.sqrt(2.0 * np.asarray(problem.r, dtype=np.float64))
    xref = np.asarray(problem.x_ref, dtype=np.float64)
    if U.ndim == 2:
        K = U.shape[1]
        R = np.empty((N, nx + nu, K))
        Ut = U.reshape(N, nu, K)
        for k in range(N):
            R[k, :nx] = (sq[:, None] * (X[k + 1] - xref).T)
            R[k, nx:] = sr[:, None] * Ut[k]
        return R.reshape(N * (nx + nu), K)
    R = np.empty((N, nx + nu))
    Ut = U.reshape(N, nu)
    for k in range(N):
        R[k, :nx] = sq * (X[k + 1] - xref)
        R[k, nx:] = sr * Ut[k]
    return R.reshape(-1)


def residual(problem, x0, U):
    """R(x0, U) of Eq. (4) for one control sequence U (n,) -> (m,), or a
    batch (n, K) -> (m, K) with the sample index fastest."""
    return residual_from_states(problem, simulate(problem, x0, U), U)


def cost_from_residual(R):
    """C = Phi(R) = 1/2 ||R||^2 (per column for a batch)."""
    R = np.asarray(R, dtype=np.float64)
    return 0.5 * np.sum(R * R, axis=0)


def cost(problem, x0, U):
    return cost_from_residual(residual(problem, x0, U))


def rollout_batch(problem, x0, U, W=None, nominal=False):
    """The rollout step of the hot path: column s evaluates U + W[:, s].
    With ``nominal`` an extra leading column evaluates U itself.
    Returns (R (m, K'), C (K',))."""
    U = np.asarray(U, dtype=np.float64)
    cols = []
    if nominal:
        cols.append(U[:, None])
    if W is not None:
        cols.append(U[:, None] + np.asarray(W, dtype=np.float64))
    Ub = np.concatenate(cols, axis=1)
    R = residual(problem, x0, Ub)
    return R, cost_from_residual(R)


def stage_cost_direct(problem, x0, U):
    """Eq. (2) evaluated from the states with the quadratic stage and
    terminal costs written out term by term (Q_N = Q, x_0 term dropped).
    Used only as a second route to check ``cost``."""
    X = simulate(problem, x0, U)
    Q = np.diag(problem.q)
    Rw = np.diag(problem.r)
    Ut = np.asarray(U, dtype=np.float64).reshape(problem.N, problem.nu)
    total = 0.0
    for k in range(problem.N):
        e = X[k + 1] - problem.x_ref
        total += e @ Q @ e + Ut[k] @ Rw @ Ut[k]
    return total
