"""Pins for the MPPI weights and step (Eqs. (5)-(8)).

Brute force in 50-digit decimal arithmetic without the min-shift, invariance
under a cost shift, the Laplace limit lambda -> 0 (argmin selection, Sec. 3)
and the uniform limit lambda -> infinity.
"""
import decimal
import itertools

import numpy as np
import pytest

from oracle import mppi


def _brute_force(W, C, lam):
    ctx = decimal.Context(prec=50)
    w = [ctx.exp(ctx.divide(-decimal.Decimal(float(c)), decimal.Decimal(float(lam)))) for c in C]
    Z = sum(w, decimal.Decimal(0))
    out = []
    for i in range(W.shape[0]):
        num = sum((decimal.Decimal(float(W[i, s])) * w[s] for s in range(W.shape[1])), decimal.Decimal(0))
        out.append(float(ctx.divide(num, Z)))
    return np.array(out), np.array([float(ctx.divide(x, Z)) for x in w])


@pytest.mark.parametrize("K,n,lam", [(2, 1, 0.3), (5, 2, 1.0), (8, 3, 0.05), (7, 3, 10.0)])
def test_step_matches_decimal_brute_force(K, n, lam):
    rng = np.random.default_rng(K * 10 + n)
    W = rng.standard_normal((n, K))
    C = rng.uniform(0.5, 3.0, K)
    dU_ref, w_ref = _brute_force(W, C, lam)
    np.testing.assert_allclose(mppi.step(W, C, lam), dU_ref, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mppi.weights(C, lam), w_ref, rtol=1e-13)


def test_enumerated_sign_set_gives_exact_expectation():
    # W = sigma * all 2^n sign vectors is a discrete distribution with mean 0,
    # covariance sigma^2 I; the empirical mean of Eq. (7) over its full
    # support equals the expectation of Eq. (5) under it.
    n, sigma, lam = 3, 0.4, 0.7
    W = sigma * np.array(list(itertools.product([-1.0, 1.0], repeat=n))).T
    C = np.array([np.sum((w - 0.1) ** 2) for w in W.T])
    expect = sum(w * np.exp(-c / lam) for w, c in zip(W.T, C)) / sum(np.exp(-c / lam) for c in C)
    np.testing.assert_allclose(mppi.step(W, C, lam), expect, rtol=1e-14)


def test_shift_invariance_and_extreme_costs():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((4, 16))
    C = rng.uniform(0, 1, 16)
    base = mppi.step(W, C, 0.2)
    # C + 1e4 is rounded to ulp(1e4) ~ 2e-12, amplified by 1/lambda in the exponent
    np.testing.assert_allclose(mppi.step(W, C + 1e4, 0.2), base, rtol=1e-9)
    # costs far beyond exp's range still give a finite step thanks to the shift
    np.testing.assert_allclose(mppi.step(W, C * 1e3 + 1e6, 200.0), base, rtol=1e-12)


def test_laplace_limit_selects_the_argmin():
    rng = np.random.default_rng(2)
    W = rng.standard_normal((3, 9))
    C = rng.uniform(0, 1, 9)
    np.testing.assert_allclose(mppi.step(W, C, 1e-8), W[:, np.argmin(C)], rtol=1e-12)


def test_uniform_limit_is_the_plain_mean():
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((3, 8))
    W = np.concatenate([Z, -Z], axis=1)
    C = rng.uniform(0, 1, 16)
    np.testing.assert_allclose(mppi.step(W, C, 1e12), np.zeros(3), atol=1e-10)


def test_nonfinite_costs_get_zero_weight():
    W = np.array([[1.0, 2.0, 3.0, 4.0]])
    C = np.array([np.nan, 1.0, np.inf, 1.0])
    w = mppi.weights(C, 1.0)
    np.testing.assert_allclose(w, [0, 0.5, 0, 0.5])
    np.testing.assert_allclose(mppi.step(W, C, 1.0), [3.0])
    with pytest.raises(mppi.NoFiniteCost):
        mppi.weights(np.array([np.nan, np.inf]), 1.0)


def _di_cost_closed_form(x0, U, N, dt, q, r):
    """Cost of the double-integrator pair (Problem IV's model, two axes)
    from the stacked closed form x_{k+1} = A^{k+1} x0 + sum_{j<=k} A^{k-j} B
    u_j, written out here with A = [[I, dt I], [0, I]], B = [[dt^2/2 I], [dt I]]
    and the stage cost q |x_{k+1}|^2 + r |u_k|^2 (x_ref = 0)."""
    I2 = np.eye(2)
    A = np.block([[I2, dt * I2], [np.zeros((2, 2)), I2]])
    B = np.vstack([0.5 * dt * dt * I2, dt * I2])
    u = np.asarray(U).reshape(N, 2)
    total = 0.0
    for k in range(N):
        x = np.linalg.matrix_power(A, k + 1) @ x0
        for j in range(k + 1):
            x = x + np.linalg.matrix_power(A, k - j) @ B @ u[j]
        total += q * x @ x + r * u[k] @ u[k]
    return total


def test_plain_mppi_laplace_limit_is_greedy_random_search():
    # With a vanishing temperature the weights of Eq. (8) collapse onto the
    # cheapest sample (the Laplace limit of Sec. 3), so Method C becomes
    # greedy random search: U <- U + W[:, argmin_s C(U + W_s)].  The greedy
    # search below evaluates its costs by the closed form above, a route
    # independent of the oracle's simulator; six iterations must agree.
    import workloads as wl
    from oracle import solvers
    N, dt = 6, 0.1
    prob = wl.double_integrator_problem(axes=2, dt=dt, N=N)
    x0 = np.array([0.7, -0.4, 0.2, 0.5])
    noise = lambda it, s: wl.gaussian_perturbations(prob.n, 16, s, 300 + it)  # noqa: E731
    U_or, _ = solvers.plain_mppi(prob, x0, np.zeros(prob.n), 6, noise, 0.3, temperature=1e-12,
                                 beta=0.9)
    U = np.zeros(prob.n)
    for it in range(6):
        W = noise(it, 0.3 * 0.9 ** (0.5 * it))
        costs = [_di_cost_closed_form(x0, U + W[:, s], N, dt, 1.0, 0.1) for s in range(W.shape[1])]
        U = U + W[:, int(np.argmin(costs))]
    np.testing.assert_allclose(U_or, U, rtol=0, atol=1e-14)


def test_plain_mppi_uniform_limit_keeps_u_with_antithetic_samples():
    # An infinite temperature gives equal weights, so the update of Eq. (7) is
    # the plain mean of W, exactly zero for antithetic pairs: U stays put.
    import workloads as wl
    from oracle import solvers
    prob = wl.double_integrator_problem(axes=2, dt=0.1, N=5)
    U0 = np.random.default_rng(4).standard_normal(prob.n)
    noise = lambda it, s: wl.gaussian_perturbations(prob.n, 32, s, 400 + it)  # noqa: E731
    U, _ = solvers.plain_mppi(prob, np.array([0.1, 0.2, 0.3, 0.4]), U0, 3, noise, 0.5,
                              temperature=1e300)
    np.testing.assert_allclose(U, U0, rtol=0, atol=1e-15)
