"""Pins for the Jacobian reconstruction of Eq. (10).

* LS form is exact on affine residuals (the linear double integrator) and
  equals the closed-form Jacobian built from the stacked system matrices.
* With antithetic pairs it is exact on any quadratic residual (Rosenbrock,
  Problem I) for any sigma, since the even terms cancel pairwise.
* On the nonlinear chain it converges to central finite differences as
  sigma -> 0 with error O(sigma^2) (the smoothing bias, Sec. 4.1).
* The MC form is unbiased on affine residuals and its error falls like
  1/sqrt(K) (Lemma 1); on a sigma-point set (Method E) it equals LS.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dynamics, jacobian, lqr, ocp, sigma_points


def _di_closed_form_jacobian(p, x0):
    A, B = dynamics.double_integrator_matrices(p.nu, p.dt)
    _, _, Gam, _ = lqr.dense_qp_solution(A, B, np.eye(p.nx), np.eye(p.nu), np.eye(p.nx), p.N, x0)
    J = np.zeros((p.m, p.n))
    sq, sr = np.sqrt(2 * p.q), np.sqrt(2 * p.r)
    for k in range(p.N):
        rows = slice(k * (p.nx + p.nu), k * (p.nx + p.nu) + p.nx)
        J[rows] = sq[:, None] * Gam[k * p.nx:(k + 1) * p.nx]
        J[k * (p.nx + p.nu) + p.nx + np.arange(p.nu), k * p.nu + np.arange(p.nu)] = sr
    return J


def test_ls_is_exact_on_the_linear_double_integrator():
    w = wl.c1()
    p = w.problem
    J_true = _di_closed_form_jacobian(p, w.x0)
    U = np.random.default_rng(0).standard_normal(p.n)
    W = wl.gaussian_perturbations(p.n, w.settings.K, 0.5, 1)
    R, _ = ocp.rollout_batch(p, w.x0, U, W, nominal=True)
    np.testing.assert_allclose(jacobian.ls(R, W), J_true, atol=1e-11 * np.abs(J_true).max())


def test_ls_exact_with_minimal_non_antithetic_sample_count():
    w = wl.c1()
    p = w.problem.with_horizon(5)
    J_true = _di_closed_form_jacobian(p, w.x0)
    W = wl.gaussian_perturbations(p.n, p.n, 0.5, 2, antithetic=False)  # K = n
    R, _ = ocp.rollout_batch(p, w.x0, np.zeros(p.n), W, nominal=True)
    np.testing.assert_allclose(jacobian.ls(R, W), J_true, atol=1e-9)
    with pytest.raises(jacobian.RankDeficient):
        jacobian.ls(R[:, :p.n], W[:, :p.n - 1])


def _rosenbrock_residual(Ub):
    u1, u2 = Ub[0], Ub[1]
    return np.stack([np.sqrt(2.0) * (1 - u1), np.sqrt(200.0) * (u2 - u1 * u1)])


@pytest.mark.parametrize("sigma", [1e-3, 0.3, 2.0])
def test_ls_exact_on_quadratic_residual_with_antithetic_pairs(sigma):
    U = np.array([0.3, -0.7])
    W = wl.gaussian_perturbations(2, 8, sigma, 5)
    R = _rosenbrock_residual(np.concatenate([U[:, None], U[:, None] + W], axis=1))
    J_true = np.array([[-np.sqrt(2.0), 0.0], [-2 * np.sqrt(200.0) * U[0], np.sqrt(200.0)]])
    np.testing.assert_allclose(jacobian.ls(R, W), J_true, atol=1e-11 * max(1, sigma ** 2) * 100)


def test_ls_converges_to_finite_differences_on_the_chain():
    prob, x0 = wl.chain_problem(n_masses=2, N=3, seed=1)
    U = 0.2 * np.random.default_rng(1).standard_normal(prob.n)
    resfun = lambda Ub: ocp.residual(prob, x0, Ub)  # noqa: E731
    J_fd = jacobian.central_fd(resfun, U, 1e-6)
    errs = []
    for sigma in (4e-2, 2e-2):
        W = wl.gaussian_perturbations(prob.n, 64, sigma, 3)
        R, _ = ocp.rollout_batch(prob, x0, U, W, nominal=True)
        errs.append(np.linalg.norm(jacobian.ls(R, W) - J_fd) / np.linalg.norm(J_fd))
    # smoothing bias is O(sigma^2): halving sigma cuts the error by ~4
    assert errs[1] < 1e-3
    assert 2.5 < errs[0] / errs[1] < 6.0, errs
    W = wl.gaussian_perturbations(prob.n, 64, 1e-3, 3)
    R, _ = ocp.rollout_batch(prob, x0, U, W, nominal=True)
    assert np.linalg.norm(jacobian.ls(R, W) - J_fd) / np.linalg.norm(J_fd) < 1e-5


def test_mc_is_unbiased_and_follows_the_lemma_1_rate():
    w = wl.c1()
    p = w.problem.with_horizon(4)
    J_true = _di_closed_form_jacobian(p, w.x0)
    sigma = 0.5
    errs = {}
    for K in (64, 1024):
        e = []
        for rep in range(40):
            W = wl.gaussian_perturbations(p.n, K, sigma, 1000 * K + rep, antithetic=False)
            R, _ = ocp.rollout_batch(p, w.x0, np.zeros(p.n), W, nominal=True)
            e.append(np.linalg.norm(jacobian.mc(R, W, sigma ** 2) - J_true))
        errs[K] = np.mean(e)
    ratio = errs[64] / errs[1024]
    assert 2.8 < ratio < 5.6, (errs, ratio)  # sqrt(1024/64) = 4


def test_mc_equals_ls_on_sigma_points():
    w = wl.c1()
    p = w.problem.with_horizon(6)
    sigma = 0.3
    W = sigma_points.symmetric_set(p.n, sigma)
    np.testing.assert_allclose(W @ W.T / W.shape[1], sigma ** 2 * np.eye(p.n), atol=1e-15)
    R, _ = ocp.rollout_batch(p, w.x0, np.ones(p.n), W, nominal=True)
    np.testing.assert_allclose(jacobian.mc(R, W, sigma ** 2), jacobian.ls(R, W), atol=1e-12)
    np.testing.assert_allclose(jacobian.ls(R, W), _di_closed_form_jacobian(p, w.x0), atol=1e-11)


def test_central_fd_on_a_polynomial():
    f = lambda Ub: np.stack([Ub[0] ** 3, Ub[0] * Ub[1]])  # noqa: E731
    U = np.array([0.5, -2.0])
    np.testing.assert_allclose(jacobian.central_fd(f, U, 1e-5),
                               [[3 * 0.25, 0.0], [-2.0, 0.5]], atol=1e-9)
