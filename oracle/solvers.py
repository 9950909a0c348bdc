"""Outer loops: Alg. 1 (GN-MPPI, Methods D and E), deterministic MPPI
(Method C) and GGN with central finite differences (Method A).  Sec. 4.3 and
Sec. 5.  Test infrastructure only.

Alg. 1 per iteration k: reconstruct J from M perturbed rollouts (Eq. (10)),
take the full GGN step (Eq. (13)), pick the step length from the set A by
parallel line search (Eqs. (14)-(15)), apply it, and shrink the covariance
Sigma <- beta Sigma.  Readings: Sigma_k = sigma_k^2 I, and since beta
multiplies the covariance the sampler's scale is
sigma_k = max(sigma_0 * beta^(k/2), sigma_min) (a floor keeps the residual
differences above rounding noise); the line-search set is {gamma^j}, j < L,
without alpha = 0, so a step is always taken.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import ggn, jacobian, mppi, ocp


@dataclass
class History:
    cost: list = field(default_factory=list)      # C(U) after each iteration
    alpha: list = field(default_factory=list)
    sigma: list = field(default_factory=list)
    grad_norm: list = field(default_factory=list)
    U: np.ndarray | None = None


def sigma_schedule(sigma0: float, beta: float, sigma_min: float, it: int) -> float:
    return max(sigma0 * beta ** (0.5 * it), sigma_min)


def gn_mppi(problem, x0, U0, iters, noise, sigma0, beta=0.9, sigma_min=1e-6,
            gamma=0.5, n_alpha=16, lm_lambda=0.0, method="ls"):
    """Alg. 1.  ``noise(it, sigma)`` returns the perturbation matrix W (n, K)
    for iteration ``it`` at scale ``sigma`` (the caller decides whether it is
    random, antithetic or a sigma-point set)."""
    U = np.asarray(U0, dtype=np.float64).copy()
    hist = History()
    alphas = ggn.step_lengths(gamma, n_alpha)
    costfun = lambda Ub: ocp.cost_from_residual(ocp.residual(problem, x0, Ub))  # noqa: E731
    for it in range(iters):
        sig = sigma_schedule(sigma0, beta, sigma_min, it)
        W = np.asarray(noise(it, sig), dtype=np.float64)
        R, _ = ocp.rollout_batch(problem, x0, U, W, nominal=True)
        if method == "ls":
            J = jacobian.ls(R, W)
        elif method == "mc":
            J = jacobian.mc(R, W, sig * sig)
        else:
            raise ValueError(method)
        r0 = R[:, 0]
        delta = ggn.direction(J, r0, lm_lambda)
        U, a, j, costs = ggn.line_search(costfun, U, delta, alphas)
        hist.cost.append(float(costs[j]))
        hist.alpha.append(float(a))
        hist.sigma.append(sig)
        hist.grad_norm.append(float(np.linalg.norm(J.T @ r0)))
    hist.U = U
    return U, hist


def plain_mppi(problem, x0, U0, iters, noise, sigma0, temperature, beta=1.0,
               sigma_min=0.0):
    """Method C: U <- U + sum_m w_m W_m / sum_m w_m, Eqs. (7)-(8)."""
    U = np.asarray(U0, dtype=np.float64).copy()
    hist = History()
    for it in range(iters):
        sig = sigma_schedule(sigma0, beta, sigma_min, it)
        W = np.asarray(noise(it, sig), dtype=np.float64)
        _, C = ocp.rollout_batch(problem, x0, U, W)
        U = mppi.update(U, W, C, temperature)
        hist.cost.append(float(ocp.cost(problem, x0, U)))
        hist.sigma.append(sig)
    hist.U = U
    return U, hist


def method_a(problem, x0, U0, iters=100, eps=1.49e-8, gamma=0.5, n_alpha=16,
             tol=1e-12):
    """Method A: GGN with a central finite-difference Jacobian, run until the
    applied step is below ``tol (1 + ||U||_inf)``.  Used to obtain the
    reference optimum C* of nonlinear workloads."""
    U = np.asarray(U0, dtype=np.float64).copy()
    hist = History()
    alphas = ggn.step_lengths(gamma, n_alpha)
    resfun = lambda Ub: ocp.residual(problem, x0, Ub)  # noqa: E731
    costfun = lambda Ub: ocp.cost_from_residual(resfun(Ub))  # noqa: E731
    for _ in range(iters):
        r0 = resfun(U)
        J = jacobian.central_fd(resfun, U, eps)
        delta = ggn.direction(J, r0)
        Unew, a, j, costs = ggn.line_search(costfun, U, delta, alphas)
        step = np.max(np.abs(Unew - U))
        U = Unew
        hist.cost.append(float(costs[j]))
        hist.alpha.append(float(a))
        hist.grad_norm.append(float(np.linalg.norm(J.T @ r0)))
        if step < tol * (1.0 + np.max(np.abs(U))):
            break
    hist.U = U
    return U, hist
