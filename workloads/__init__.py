"""Seeded synthetic inputs for the Gauss-Newton accelerated MPPI hot path.

This module holds problem *data* only: sizes, diagonal weights, initial and
reference states, hyper-parameters and Gaussian perturbation matrices drawn
with numpy's PCG64 generator.  None of the method's arithmetic lives here (no
dynamics, residuals, weights, Jacobians or solves), so both the CPU oracle and
the GPU path can take their inputs from it without sharing any computation.

Workloads (paper: direct single-shooting OCP of Sec. 2, Eqs. (1)-(4)):

* ``c1`` -- the linear double integrator of Problem IV (Sec. 5) as a pair of
  axes: nx=4, nu=2, dt=0.1, N=20, K=256, sigma=0.5, Q=I, R=0.1 I, FP64.
* ``c2`` -- a planar chain of 16 unit point masses joined by cubic springs
  (k_lin=1, k_cub=0.5), end-mass velocity input, RK4 with dt=0.05, N=50,
  K=4096, sigma=0.3, FP32.  It stands in for the paper's RK4-discretised
  nonlinear pendulum of Problem V, whose model is given only by citation.
* ``c4`` -- the same chain at N=66, K=8192 (precision-split workload).
* ``c3`` -- batches of independent chain instances of uneven size.
* warm-start data -- initial states of the chain instance drawn like its x0
  (``chain_initial_states``), solved by GN-MPPI to give (x0, U*) pairs.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

MODEL_DOUBLE_INTEGRATOR = 1
MODEL_CHAIN = 2


@dataclass(frozen=True)
class Problem:
    """Direct single-shooting OCP data (paper Sec. 2).

    State order: double integrator (p_1..p_d, v_1..v_d); chain
    (p_1x, p_1y, ..., p_Mx, p_My, v_1x, v_1y, ..., v_Mx, v_My).
    ``q`` and ``r`` are the diagonals of the stage weights Q and R; ``x_ref``
    is the tracking target.  Residual rows per step k are the nx state rows of
    x_{k+1} followed by the nu input rows of u_k.
    """

    model: int
    nx: int
    nu: int
    N: int
    dt: float
    q: np.ndarray
    r: np.ndarray
    x_ref: np.ndarray
    n_masses: int = 0
    k_lin: float = 0.0
    k_cub: float = 0.0
    mass: float = 1.0

    @property
    def n(self) -> int:
        return self.N * self.nu

    @property
    def m(self) -> int:
        return self.N * (self.nx + self.nu)

    def with_horizon(self, N: int) -> "Problem":
        return dataclasses.replace(self, N=N)


@dataclass(frozen=True)
class SolverSettings:
    """Hyper-parameters of Alg. 1 (and of plain MPPI, Eqs. (7)-(8))."""

    iters: int
    K: int
    sigma0: float
    beta: float = 0.9
    sigma_min: float = 1e-6
    gamma: float = 0.5
    n_alpha: int = 16
    lm_lambda: float = 0.0
    antithetic: bool = True
    jacobian: str = "ls"  # "ls" (default reading) or "mc" (literal Eq. (10))
    # precision of the S = dR W^T contraction for float32 workloads: "native"
    # (FP32 MFMA), "bf16x3" (hi/lo BF16 split, FP32-level error) or "bf16"
    # (the precision split: BF16 operands, FP32 accumulation)
    contraction: str = "native"
    temperature: float = 1.0  # MPPI lambda_k for the plain-MPPI comparator
    mppi_sigma0: float = 0.0  # plain-MPPI sampling scale (0 -> sigma0)
    mppi_beta: float = 1.0


@dataclass(frozen=True)
class Workload:
    name: str
    problem: Problem
    x0: np.ndarray
    settings: SolverSettings
    dtype: str  # "f32" or "f64"
    description: str = ""
    noise_seed: int = 1


# ---------------------------------------------------------------------------
# problem constructors (data only)
# ---------------------------------------------------------------------------

def double_integrator_problem(axes: int = 2, dt: float = 0.1, N: int = 20,
                              q: float = 1.0, r: float = 0.1) -> Problem:
    nx, nu = 2 * axes, axes
    return Problem(model=MODEL_DOUBLE_INTEGRATOR, nx=nx, nu=nu, N=N, dt=dt,
                   q=np.full(nx, q), r=np.full(nu, r), x_ref=np.zeros(nx))


def chain_rest_pose(n_masses: int, end_point) -> np.ndarray:
    """Equilibrium of the zero-rest-length spring chain: masses evenly spaced
    on the segment from the fixed anchor (origin) to ``end_point``, at rest."""
    e = np.asarray(end_point, dtype=np.float64)
    pos = np.outer(np.arange(1, n_masses + 1) / n_masses, e).reshape(-1)
    return np.concatenate([pos, np.zeros(2 * n_masses)])


def chain_problem(n_masses: int = 16, N: int = 50, dt: float = 0.05,
                  k_lin: float = 1.0, k_cub: float = 0.5, mass: float = 1.0,
                  q: float = 1.0, r: float = 0.1, seed: int = 0) -> tuple[Problem, np.ndarray]:
    """Chain instance: reference = rest pose for e_ref ~ U[-1,1]^2; initial
    state = rest pose for e0 ~ U[-1,1]^2 with U[-0.1,0.1] jitter on the free
    masses' positions and velocities; the end mass starts at rest."""
    rng = np.random.default_rng(seed)
    e_ref = rng.uniform(-1.0, 1.0, 2)
    e0 = rng.uniform(-1.0, 1.0, 2)
    M = n_masses
    x_ref = chain_rest_pose(M, e_ref)
    x0 = chain_rest_pose(M, e0)
    free = 2 * (M - 1)
    x0[:free] += rng.uniform(-0.1, 0.1, free)
    x0[2 * M:2 * M + free] += rng.uniform(-0.1, 0.1, free)
    nx = 4 * M
    prob = Problem(model=MODEL_CHAIN, nx=nx, nu=2, N=N, dt=dt, q=np.full(nx, q),
                   r=np.full(2, r), x_ref=x_ref, n_masses=M, k_lin=k_lin,
                   k_cub=k_cub, mass=mass)
    return prob, x0


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def c1() -> Workload:
    prob = double_integrator_problem(axes=2, dt=0.1, N=20)
    x0 = np.random.default_rng(0).uniform(-1.0, 1.0, 4)
    st = SolverSettings(iters=20, K=256, sigma0=0.5, beta=0.9, sigma_min=1e-6,
                        gamma=0.5, n_alpha=16, temperature=0.05, mppi_sigma0=0.5,
                        mppi_beta=0.95)
    return Workload("c1", prob, x0, st, "f64",
                    "double-integrator pair nx=4 nu=2 dt=0.1 N=20 K=256 sigma=0.5 fp64")


def c2() -> Workload:
    prob, x0 = chain_problem(n_masses=16, N=50, dt=0.05, seed=0)
    st = SolverSettings(iters=50, K=4096, sigma0=0.3, beta=0.9, sigma_min=1e-3,
                        gamma=0.5, n_alpha=16, temperature=0.05, mppi_sigma0=0.3,
                        mppi_beta=0.98, contraction="bf16x3")
    return Workload("c2", prob, x0, st, "f32",
                    "chain16 cubic springs RK4 nx=64 nu=2 dt=0.05 N=50 K=4096 sigma=0.3 fp32")


def c4() -> Workload:
    prob, x0 = chain_problem(n_masses=16, N=66, dt=0.05, seed=0)
    st = SolverSettings(iters=50, K=8192, sigma0=0.3, beta=0.9, sigma_min=1e-3,
                        gamma=0.5, n_alpha=16, contraction="bf16")
    return Workload("c4", prob, x0, st, "f32",
                    "chain16 RK4 N=66 m=4356 n=132 K=8192 precision split")


def small_chain(n_masses: int = 3, N: int = 6, seed: int = 0) -> Workload:
    """A chain small enough for pure-CPU checks that still spans several
    GPU tiles when K is a few hundred."""
    prob, x0 = chain_problem(n_masses=n_masses, N=N, dt=0.05, seed=seed)
    st = SolverSettings(iters=5, K=256, sigma0=0.3, sigma_min=1e-3)
    return Workload(f"chain{n_masses}_N{N}", prob, x0, st, "f32")


WORKLOADS = {"c1": c1, "c2": c2, "c4": c4}


def get(name: str) -> Workload:
    return WORKLOADS[name]()


# ---------------------------------------------------------------------------
# random inputs
# ---------------------------------------------------------------------------

def gaussian_perturbations(n: int, K: int, sigma: float, seed: int,
                           antithetic: bool = True) -> np.ndarray:
    """W in R^{n x K} (sample index fastest): i.i.d. N(0, sigma^2) columns;
    with ``antithetic`` the second half of the columns is the negated first
    half (W[:, s + K/2] = -W[:, s])."""
    rng = np.random.default_rng(seed)
    if antithetic:
        if K % 2:
            raise ValueError("antithetic sampling needs an even K")
        Z = rng.standard_normal((n, K // 2))
        return sigma * np.concatenate([Z, -Z], axis=1)
    return sigma * rng.standard_normal((n, K))


def chain_initial_states(count: int, seed: int, n_masses: int = 16) -> np.ndarray:
    """Initial states drawn like the chain instance's x0 (rest pose for
    e0 ~ U[-1,1]^2, U[-0.1,0.1] jitter on the free masses' positions and
    velocities, end mass at rest): the inputs of the warm-start data set,
    ``count`` x 4 M."""
    rng = np.random.default_rng(seed)
    M = n_masses
    free = 2 * (M - 1)
    out = np.empty((count, 4 * M))
    for i in range(count):
        x0 = chain_rest_pose(M, rng.uniform(-1.0, 1.0, 2))
        x0[:free] += rng.uniform(-0.1, 0.1, free)
        x0[2 * M:2 * M + free] += rng.uniform(-0.1, 0.1, free)
        out[i] = x0
    return out


def random_controls(n: int, scale: float, seed: int) -> np.ndarray:
    return scale * np.random.default_rng(seed).standard_normal(n)


def batch_instances(count: int, seed: int = 0, masses=(4, 16), horizons=(20, 80),
                    sample_counts=(512, 1024, 2048, 4096)):
    """Uneven batch of chain MPC instances (masses in [4,16], N in [20,80],
    K from ``sample_counts``), each with its own seeded initial and reference
    state."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        M = int(rng.integers(masses[0], masses[1] + 1))
        N = int(rng.integers(horizons[0], horizons[1] + 1))
        K = int(rng.choice(sample_counts))
        prob, x0 = chain_problem(n_masses=M, N=N, dt=0.05, seed=int(rng.integers(1 << 31)))
        out.append((prob, x0, K))
    return out
