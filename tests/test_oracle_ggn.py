"""Pins for the GGN step (Eq. (13)), line search (Eqs. (14)-(15)), the LQR
reference and the outer loops of Alg. 1 and Methods A/C."""
import numpy as np
import pytest

import workloads as wl
from oracle import dynamics, ggn, jacobian, lqr, ocp, solvers


def _c1_reference():
    w = wl.c1()
    p = w.problem
    A, B = dynamics.double_integrator_matrices(2, p.dt)
    Q, R = np.diag(p.q), np.diag(p.r)
    return w, lqr.riccati_solution(A, B, Q, R, Q, p.N, w.x0), lqr.dense_qp_solution(A, B, Q, R, Q, p.N, w.x0)


def test_riccati_and_dense_qp_agree_and_match_the_cost():
    w, (U1, c1), (U2, c2, _, _) = _c1_reference()
    np.testing.assert_allclose(U1, U2, atol=1e-12)
    assert abs(c1 - c2) < 1e-12 * c1
    assert abs(ocp.cost(w.problem, w.x0, U1) - c1) < 1e-12 * c1


def test_paper_size_problem_iv_also_agrees():
    # Problem IV as printed: x0 in R^2 (one axis), N = 50
    A, B = dynamics.double_integrator_matrices(1, 0.1)
    Q, R = np.eye(2), 0.1 * np.eye(1)
    x0 = np.array([1.0, -0.5])
    U1, c1 = lqr.riccati_solution(A, B, Q, R, Q, 50, x0)
    U2, c2, _, _ = lqr.dense_qp_solution(A, B, Q, R, Q, 50, x0)
    np.testing.assert_allclose(U1, U2, atol=1e-11)
    assert abs(c1 - c2) < 1e-11 * c1


def test_one_gn_mppi_iteration_hits_the_lqr_optimum():
    w, (Ustar, cstar), _ = _c1_reference()
    p = w.problem
    noise = lambda it, s: wl.gaussian_perturbations(p.n, w.settings.K, s, 10 + it)  # noqa: E731
    U, hist = solvers.gn_mppi(p, w.x0, np.zeros(p.n), 1, noise, w.settings.sigma0)
    assert abs(hist.cost[0] - cstar) / cstar < 1e-10
    np.testing.assert_allclose(U, Ustar, atol=1e-9)
    assert hist.alpha[0] == 1.0


def test_direction_equals_least_squares_minimiser():
    rng = np.random.default_rng(0)
    J = rng.standard_normal((30, 7))
    r0 = rng.standard_normal(30)
    d_ls = np.linalg.lstsq(J, -r0, rcond=None)[0]
    np.testing.assert_allclose(ggn.direction(J, r0), d_ls, atol=1e-12)
    lam = 0.7
    Ja = np.vstack([J, np.sqrt(lam) * np.eye(7)])
    d_reg = np.linalg.lstsq(Ja, np.concatenate([-r0, np.zeros(7)]), rcond=None)[0]
    np.testing.assert_allclose(ggn.direction(J, r0, lam), d_reg, atol=1e-12)


def test_direction_rejects_singular_normal_matrix():
    J = np.zeros((5, 3))
    with pytest.raises(ggn.NotPositiveDefinite):
        ggn.direction(J, np.ones(5))


def test_line_search_picks_first_minimum():
    alphas = ggn.step_lengths(0.5, 6)
    np.testing.assert_allclose(alphas, [1, 0.5, 0.25, 0.125, 0.0625, 0.03125])
    # convex quadratic along the line with minimiser at alpha = 0.25
    cost = lambda Ub: (Ub[0] - 0.25) ** 2  # noqa: E731
    U, a, j, costs = ggn.line_search(cost, np.zeros(1), np.ones(1), alphas)
    assert (a, j) == (0.25, 2)
    # ties resolve to the largest step
    flat = lambda Ub: np.zeros(Ub.shape[1])  # noqa: E731
    assert ggn.line_search(flat, np.zeros(1), np.ones(1), alphas)[2] == 0
    # NaN candidates are never chosen
    nanc = lambda Ub: np.where(Ub[0] > 0.9, np.nan, Ub[0])  # noqa: E731
    assert ggn.line_search(nanc, np.zeros(1), np.ones(1), alphas)[2] == 5


def test_gn_mppi_solves_rosenbrock_from_the_origin():
    # Problem I as a "rollout" of a 2-variable inner function
    class P:
        pass
    resfun = lambda Ub: np.stack([np.sqrt(2.0) * (1 - Ub[0]), np.sqrt(200.0) * (Ub[1] - Ub[0] ** 2)])  # noqa: E731
    U = np.zeros(2)
    alphas = ggn.step_lengths(0.5, 16)
    for it in range(40):
        W = wl.gaussian_perturbations(2, 16, 0.3 * 0.9 ** (0.5 * it), it)
        R = resfun(np.concatenate([U[:, None], U[:, None] + W], axis=1))
        J = jacobian.ls(R, W)
        d = ggn.direction(J, R[:, 0])
        U, *_ = ggn.line_search(lambda Ub: 0.5 * np.sum(resfun(Ub) ** 2, axis=0), U, d, alphas)
    np.testing.assert_allclose(U, [1.0, 1.0], atol=1e-8)


@pytest.mark.slow
def test_gn_mppi_reaches_method_a_optimum_on_a_small_chain():
    w = wl.small_chain(n_masses=3, N=8)
    p = w.problem
    _, ha = solvers.method_a(p, w.x0, np.zeros(p.n), iters=60)
    noise = lambda it, s: wl.gaussian_perturbations(p.n, 64, s, 50 + it)  # noqa: E731
    _, hg = solvers.gn_mppi(p, w.x0, np.zeros(p.n), 25, noise, 0.3, sigma_min=1e-4)
    cstar = ha.cost[-1]
    assert ha.grad_norm[-1] < 1e-6 * (1 + cstar)
    assert (hg.cost[-1] - cstar) / cstar < 1e-6
    # plain MPPI decreases the cost but stays far slower than GN-MPPI
    _, hm = solvers.plain_mppi(p, w.x0, np.zeros(p.n), 25, noise, 0.3, temperature=0.05)
    assert hm.cost[-1] < ocp.cost(p, w.x0, np.zeros(p.n))
    assert hm.cost[-1] > hg.cost[-1]
