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
