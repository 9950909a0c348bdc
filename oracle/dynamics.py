"""Discrete-time dynamics x_{k+1} = f(x_k, u_k) behind the simulator F of
Eq. (1) (Sec. 2).  Test infrastructure only (see the package docstring).

All functions are batched over leading axes: ``x`` has shape (..., nx) and
``u`` shape (..., nu).  Float64 throughout.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Problem IV: linear double integrator (Sec. 5)
# ---------------------------------------------------------------------------

def double_integrator_matrices(axes: int, dt: float):
    """(A, B) of x_{k+1} = A x_k + B u_k for ``axes`` independent double
    integrators with the input held constant over the step (exact
    zero-order hold): p+ = p + dt v + dt^2/2 u, v+ = v + dt u.  State order
    (p_1..p_d, v_1..v_d)."""
    I = np.eye(axes)
    Z = np.zeros((axes, axes))
    A = np.block([[I, dt * I], [Z, I]])
    B = np.vstack([0.5 * dt * dt * I, dt * I])
    return A, B


def double_integrator_step(x, u, dt: float):
    d = u.shape[-1]
    p, v = x[..., :d], x[..., d:]
    return np.concatenate([p + dt * v + 0.5 * dt * dt * u, v + dt * u], axis=-1)


# ---------------------------------------------------------------------------
# Planar spring chain, RK4 with the input held over the step (as Problem V)
# ---------------------------------------------------------------------------

def chain_rhs(x, u, n_masses: int, k_lin: float, k_cub: float, mass: float):
    """Continuous-time right-hand side of the chain.

    Masses i = 1..M in the plane, anchor p_0 = 0 fixed.  Link i joins
    p_{i-1} and p_i with zero rest length and force
    T_i = (k_lin + k_cub |d_i|^2) d_i, d_i = p_i - p_{i-1}.  Free masses
    (i < M) obey m a_i = T_{i+1} - T_i.  The end mass is driven kinematically
    by the input: dp_M/dt = u, and its velocity slot has zero derivative (it
    is overwritten with u after each step, see ``chain_step``).
    """
    M = n_masses
    lead = x.shape[:-1]
    P = x[..., : 2 * M].reshape(lead + (M, 2))
    V = x[..., 2 * M:].reshape(lead + (M, 2))
    prev = np.concatenate([np.zeros(lead + (1, 2)), P[..., :-1, :]], axis=-2)
    D = P - prev
    T = (k_lin + k_cub * np.sum(D * D, axis=-1, keepdims=True)) * D
    acc = np.zeros_like(P)
    acc[..., :-1, :] = (T[..., 1:, :] - T[..., :-1, :]) / mass
    pdot = V.copy()
    pdot[..., -1, :] = u
    return np.concatenate([pdot.reshape(lead + (2 * M,)), acc.reshape(lead + (2 * M,))], axis=-1)


def rk4_step(rhs, x, u, h: float):
    """Classical explicit Runge-Kutta of order 4 with u constant over [t, t+h]."""
    s1 = rhs(x, u)
    s2 = rhs(x + 0.5 * h * s1, u)
    s3 = rhs(x + 0.5 * h * s2, u)
    s4 = rhs(x + h * s3, u)
    return x + (h / 6.0) * (s1 + 2.0 * s2 + 2.0 * s3 + s4)


def chain_step(x, u, dt: float, n_masses: int, k_lin: float, k_cub: float, mass: float):
    M = n_masses
    rhs = lambda xx, uu: chain_rhs(xx, uu, M, k_lin, k_cub, mass)  # noqa: E731
    xn = rk4_step(rhs, x, u, dt)
    xn[..., 4 * M - 2: 4 * M] = u  # end-mass velocity equals the commanded velocity
    return xn


def step(problem, x, u):
    """One step of the problem's dynamics (dispatch on ``problem.model``)."""
    if problem.model == 1:
        return double_integrator_step(x, u, problem.dt)
    if problem.model == 2:
        return chain_step(x, u, problem.dt, problem.n_masses, problem.k_lin,
                          problem.k_cub, problem.mass)
    raise ValueError(f"unknown model {problem.model}")
