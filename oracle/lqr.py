"""Exact optimum of the linear-quadratic Problem IV (Sec. 5) by two routes.
Test infrastructure only.

The problem is a quadratic program ("could be solved in a single Newton
step", Sec. 5 discussion), so one GGN step with an exact Jacobian and unit
step length must land on this optimum.  Cost convention as in ``ocp``: stage
cost x_k^T Q x_k + u_k^T R u_k for k = 0..N-1 plus x_N^T Q_N x_N, reported
without the constant x_0^T Q x_0 term.
"""
from __future__ import annotations

import numpy as np


def riccati(A, B, Q, R, QN, N):
    """Backward recursion P_N = Q_N, G_k = (R + B^T P_{k+1} B)^{-1} B^T P_{k+1} A,
    P_k = Q + A^T P_{k+1} (A - B G_k).  Returns (P_0, [G_0..G_{N-1}])."""
    P = np.array(QN, dtype=np.float64)
    gains = [None] * N
    for k in range(N - 1, -1, -1):
        Gk = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        P = Q + A.T @ P @ (A - B @ Gk)
        gains[k] = Gk
    return P, gains


def riccati_solution(A, B, Q, R, QN, N, x0):
    """Optimal controls u_k = -G_k x_k and the optimal cost (x_0 term removed)."""
    P0, gains = riccati(A, B, Q, R, QN, N)
    x = np.asarray(x0, dtype=np.float64)
    U = []
    for k in range(N):
        u = -gains[k] @ x
        U.append(u)
        x = A @ x + B @ u
    x0 = np.asarray(x0, dtype=np.float64)
    cstar = float(x0 @ P0 @ x0 - x0 @ Q @ x0)
    return np.concatenate(U), cstar


def dense_qp_solution(A, B, Q, R, QN, N, x0):
    """Second route: stack x_{1..N} = Lam x0 + Gam U and solve the normal
    equations (Gam^T Qbar Gam + Rbar) U = -Gam^T Qbar Lam x0."""
    nx, nu = B.shape
    Lam = np.zeros((N * nx, nx))
    Gam = np.zeros((N * nx, N * nu))
    Ak = np.eye(nx)
    powers = [np.eye(nx)]
    for k in range(N):
        Ak = A @ Ak
        powers.append(Ak)
        Lam[k * nx:(k + 1) * nx] = Ak
    for k in range(N):          # block row: x_{k+1}
        for j in range(k + 1):  # depends on u_j
            Gam[k * nx:(k + 1) * nx, j * nu:(j + 1) * nu] = powers[k - j] @ B
    Qbar = np.zeros((N * nx, N * nx))
    for k in range(N):
        Qbar[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = QN if k == N - 1 else Q
    Rbar = np.kron(np.eye(N), R)
    x0 = np.asarray(x0, dtype=np.float64)
    H = Gam.T @ Qbar @ Gam + Rbar
    U = -np.linalg.solve(H, Gam.T @ Qbar @ Lam @ x0)
    X = Lam @ x0 + Gam @ U
    cstar = float(X @ Qbar @ X + U @ Rbar @ U)
    return U, cstar, Gam, Lam
