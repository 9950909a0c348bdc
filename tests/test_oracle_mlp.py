"""Pins of the warm-start network oracle (oracle/mlp.py) against what the
definitions fix independently of its own formulas:

* bfloat16 rounding: hand-worked bit patterns (ties to even) and torch's own
  float32 -> bfloat16 conversion;
* GELU: closed-form values (gelu(0) = 0, the z Phi(z) tails, Phi(1) from
  the normal table) and a central difference of gelu for gelu';
* backpropagation: central finite differences of the loss in float64 on a
  tiny network, every parameter;
* Adam: the closed form of the first step, lr * g / (|g| + eps).
"""
import math

import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_bit_patterns():
    one = 1.0
    ulp = 2.0 ** -7  # bfloat16 spacing just above 1
    assert mlp.bf16(one + ulp / 2)[()] == one            # tie -> even (1.0)
    assert mlp.bf16(one + 3 * ulp / 2)[()] == one + 2 * ulp  # tie -> even (1 + 2 ulp)
    assert mlp.bf16(one + ulp / 2 + 2.0 ** -20)[()] == one + ulp
    assert mlp.bf16(-3.0)[()] == -3.0
    assert mlp.bf16(0.1)[()] == 0.10009765625
    assert np.isnan(mlp.bf16(np.nan))


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(20000) * np.exp(np.random.default_rng(1).uniform(-20, 20, 20000))
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_gelu_values_and_derivative():
    assert mlp.gelu(0.0) == 0.0
    # Phi(1) = 0.8413447460685429 (standard normal table)
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(-1.0) + 1.0 - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-15 and abs(mlp.gelu(-10.0)) < 1e-20
    z = np.linspace(-4, 4, 33)
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-9)
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15


def test_backward_matches_central_differences():
    I, H, O, B = 3, 5, 4, 7
    rng = np.random.default_rng(3)
    p = 0.5 * rng.standard_normal(mlp.param_count(I, H, O))
    X = rng.standard_normal((B, I))
    T = rng.standard_normal((B, O))
    L, g = mlp.backward(p, X, T, I, H, O, bf16_ops=False)
    assert abs(L - mlp.loss(mlp.forward(p, X, I, H, O, bf16_ops=False)[0], T)) < 1e-15
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp = mlp.loss(mlp.forward(p + e, X, I, H, O, bf16_ops=False)[0], T)
        lm = mlp.loss(mlp.forward(p - e, X, I, H, O, bf16_ops=False)[0], T)
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-10)


def test_pack_unpack_layout():
    I, H, O = 2, 3, 4
    p = np.arange(mlp.param_count(I, H, O), dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, I, H, O)
    assert W1.shape == (3, 2) and W1[1, 0] == 2 and b1[0] == 6 and W2[0, 0] == 9
    assert b2[0] == 18 and W3.shape == (4, 3) and W3[0, 0] == 21 and b3[-1] == p[-1]
    np.testing.assert_array_equal(mlp.pack([W1, b1, W2, b2, W3, b3]), p)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    lr, eps = 1e-2, 1e-8
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, lr, eps=eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    assert math.isclose(p1[3], 1.0)


def test_adam_bias_correction_with_a_constant_gradient():
    # With the same gradient g at every step, m_t = (1 - beta1^t) g and
    # v_t = (1 - beta2^t) g^2, so the bias-corrected moments are exactly g and
    # g^2 at every t and each step moves by lr g / (|g| + eps): after T steps
    # p_T = p_0 - T lr g / (|g| + eps).  A correction by (1 - beta)^t, or none,
    # agrees with this only at t = 1.
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    p0 = np.array([1.0, -1.0, 0.5, 2.0])
    lr, eps, T = 1e-3, 1e-8, 25
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, T + 1):
        p, m, v = mlp.adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=eps)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(m, (1 - 0.9 ** T) * g, rtol=1e-12)
    np.testing.assert_allclose(v, (1 - 0.999 ** T) * g * g, rtol=1e-12)
