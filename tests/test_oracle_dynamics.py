"""Pins for the oracle's simulator (Eq. (1)) and cost (Eqs. (2), (4)).

Each check uses a route other than the oracle's own formula: the matrix
exponential of the continuous-time system, the Taylor polynomial of RK4 on a
linear ODE, a high-accuracy ODE integrator, a hand-derived two-mass force
law, equilibria and a term-by-term cost.
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import workloads as wl
from oracle import dynamics, lqr, ocp


def test_double_integrator_is_exact_zero_order_hold():
    # continuous system d/dt (p, v, u) = (v, u, 0); expm gives the exact
    # transition over dt with u held constant.
    d, dt = 2, 0.1
    Mc = np.zeros((3 * d, 3 * d))
    Mc[:d, d:2 * d] = np.eye(d)
    Mc[d:2 * d, 2 * d:] = np.eye(d)
    E = scipy.linalg.expm(Mc * dt)
    A_ref, B_ref = E[:2 * d, :2 * d], E[:2 * d, 2 * d:]
    A, B = dynamics.double_integrator_matrices(d, dt)
    np.testing.assert_allclose(A, A_ref, atol=1e-14)
    np.testing.assert_allclose(B, B_ref, atol=1e-14)
    rng = np.random.default_rng(3)
    x, u = rng.standard_normal((5, 2 * d)), rng.standard_normal((5, d))
    np.testing.assert_allclose(dynamics.double_integrator_step(x, u, dt),
                               x @ A_ref.T + u @ B_ref.T, atol=1e-14)


def test_double_integrator_rollout_matches_stacked_closed_form():
    w = wl.c1()
    p = w.problem
    A, B = dynamics.double_integrator_matrices(2, p.dt)
    U = np.random.default_rng(1).standard_normal(p.n)
    _, _, Gam, Lam = lqr.dense_qp_solution(A, B, np.eye(4), np.eye(2), np.eye(4), p.N, w.x0)
    X = ocp.simulate(p, w.x0, U)
    np.testing.assert_allclose(X[1:].reshape(-1), Lam @ w.x0 + Gam @ U, atol=1e-12)


def _chain_linear_matrices(M, k_lin, mass):
    """Continuous-time (A, B) of the chain with k_cub = 0, built from the
    chain's stiffness (graph Laplacian) matrix rather than from the force
    routine: free mass i feels k (p_{i+1} - 2 p_i + p_{i-1}); the end mass
    moves with the input."""
    nx = 4 * M
    Kst = np.zeros((M, M))
    for i in range(M - 1):            # free masses 0..M-2 (0-based)
        Kst[i, i] = -2.0 * k_lin / mass
        if i > 0:
            Kst[i, i - 1] = k_lin / mass
        Kst[i, i + 1] = k_lin / mass
    A = np.zeros((nx, nx))
    B = np.zeros((nx, 2))
    I2 = np.eye(2)
    for i in range(M - 1):
        A[2 * i:2 * i + 2, 2 * M + 2 * i:2 * M + 2 * i + 2] = I2      # dp = v
        for j in range(M):
            A[2 * M + 2 * i:2 * M + 2 * i + 2, 2 * j:2 * j + 2] = Kst[i, j] * I2
    B[2 * (M - 1):2 * M, :] = I2                                  # dp_M = u
    return A, B


@pytest.mark.parametrize("M", [1, 2, 5, 16])
def test_chain_rk4_linear_case_equals_taylor_polynomial(M):
    k_lin, mass, h = 1.3, 0.7, 0.05
    A, B = _chain_linear_matrices(M, k_lin, mass)
    nx = 4 * M
    hA = h * A
    I = np.eye(nx)
    Phi = I + hA + hA @ hA / 2 + hA @ hA @ hA / 6 + hA @ hA @ hA @ hA / 24
    Gam = h * (I + hA / 2 + hA @ hA / 6 + hA @ hA @ hA / 24) @ B
    rng = np.random.default_rng(M)
    x, u = rng.standard_normal(nx), rng.standard_normal(2)
    expect = Phi @ x + Gam @ u
    expect[4 * M - 2:] = u
    got = dynamics.chain_step(x, u, h, M, k_lin, 0.0, mass)
    np.testing.assert_allclose(got, expect, atol=1e-13)


def test_chain_rk4_has_fifth_order_local_error():
    M, k_lin, k_cub, mass = 4, 1.0, 0.5, 1.0
    rng = np.random.default_rng(7)
    x = rng.uniform(-0.6, 0.6, 4 * M)
    u = rng.uniform(-0.5, 0.5, 2)
    rhs = lambda t, y: dynamics.chain_rhs(y, u, M, k_lin, k_cub, mass)  # noqa: E731
    errs = []
    for h in (0.2, 0.1):
        ref = scipy.integrate.solve_ivp(rhs, (0, h), x, rtol=1e-13, atol=1e-14, method="DOP853").y[:, -1]
        ref[4 * M - 2:] = u
        errs.append(np.linalg.norm(dynamics.chain_step(x, u, h, M, k_lin, k_cub, mass) - ref))
    ratio = errs[0] / errs[1]
    assert 22.0 < ratio < 45.0, (errs, ratio)  # 2^5 = 32 for a 4th-order method


def test_chain_two_mass_force_law_by_hand():
    k_lin, k_cub, mass = 1.0, 0.5, 2.0
    rng = np.random.default_rng(11)
    for _ in range(5):
        p1, p2, v1, v2 = rng.standard_normal((4, 2))
        u = rng.standard_normal(2)
        d1, d2 = p1, p2 - p1
        T1 = (k_lin + k_cub * (d1 @ d1)) * d1
        T2 = (k_lin + k_cub * (d2 @ d2)) * d2
        expect = np.concatenate([v1, u, (T2 - T1) / mass, [0.0, 0.0]])
        x = np.concatenate([p1, p2, v1, v2])
        np.testing.assert_allclose(dynamics.chain_rhs(x, u, 2, k_lin, k_cub, mass), expect, atol=1e-14)


def test_chain_single_mass_is_kinematic():
    x = np.array([0.3, -0.2, 5.0, 6.0])
    u = np.array([0.7, -1.1])
    got = dynamics.chain_step(x, u, 0.05, 1, 1.0, 0.5, 1.0)
    np.testing.assert_allclose(got, [0.3 + 0.05 * 0.7, -0.2 - 0.05 * 1.1, 0.7, -1.1], atol=1e-15)


def test_chain_rest_pose_is_a_fixed_point():
    prob, _ = wl.chain_problem(n_masses=16, N=10, seed=4)
    X = ocp.simulate(prob, prob.x_ref, np.zeros(prob.n))
    np.testing.assert_allclose(X, np.broadcast_to(prob.x_ref, X.shape), atol=1e-13)
    assert ocp.cost(prob, prob.x_ref, np.zeros(prob.n)) < 1e-24


@pytest.mark.parametrize("name", ["c1", "chain"])
def test_cost_is_half_squared_residual_and_matches_stage_sum(name):
    if name == "c1":
        w = wl.c1()
    else:
        w = wl.small_chain(n_masses=4, N=7)
    p = w.problem
    U = 0.3 * np.random.default_rng(5).standard_normal(p.n)
    r = ocp.residual(p, w.x0, U)
    assert r.shape == (p.m,)
    np.testing.assert_allclose(ocp.cost(p, w.x0, U), ocp.stage_cost_direct(p, w.x0, U), rtol=1e-13)


def test_batched_residual_equals_per_column():
    w = wl.small_chain(n_masses=3, N=5)
    p = w.problem
    rng = np.random.default_rng(2)
    U = rng.standard_normal(p.n) * 0.2
    W = wl.gaussian_perturbations(p.n, 6, 0.3, 9)
    R, C = ocp.rollout_batch(p, w.x0, U, W, nominal=True)
    assert R.shape == (p.m, 7)
    np.testing.assert_allclose(R[:, 0], ocp.residual(p, w.x0, U), atol=1e-14)
    for s in range(6):
        np.testing.assert_allclose(R[:, s + 1], ocp.residual(p, w.x0, U + W[:, s]), atol=1e-14)
        np.testing.assert_allclose(C[s + 1], ocp.cost(p, w.x0, U + W[:, s]), rtol=1e-14)
    # residual rows: the u-block of step k is sqrt(2 r) u_k
    Ut = U.reshape(p.N, p.nu)
    for k in range(p.N):
        np.testing.assert_allclose(R[k * (p.nx + p.nu) + p.nx:(k + 1) * (p.nx + p.nu), 0],
                                   np.sqrt(2 * p.r) * Ut[k], atol=1e-15)
