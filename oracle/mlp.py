"""Warm-start network: a three-layer perceptron with GELU activations, its
squared-error loss, backpropagated gradients and the Adam update.  Test
infrastructure only.

This is not part of the paper's method: the learned warm start is an
extension in which GN-MPPI starts from a network's proposal U0(x0) instead
of from zero (the solver of Alg. 1 is unchanged).  Definitions written out
here:

* layer l:  z_l = a_{l-1} W_l^T + b_l,  a_l = gelu(z_l) for the two hidden
  layers, the output layer is linear;  gelu(z) = z Phi(z) with Phi the
  standard normal CDF, Phi(z) = (1 + erf(z / sqrt 2)) / 2;
* loss L = 1 / (2 B O) sum_{b,o} (y_bo - t_bo)^2 over a batch of B rows and
  O outputs;
* gradients by the chain rule, layer by layer (dL/dz = dL/da * gelu'(z),
  gelu'(z) = Phi(z) + z phi(z));
* Adam (Kingma and Ba, 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Mixed precision as the GPU computes it: every matrix-product operand is
rounded to bfloat16 (round to nearest, ties to even) and the products are
summed exactly (float64 here, float32 on the device); everything else stays
in float64.  With ``bf16=False`` the same functions give the plain float64
network, which the finite-difference pins check.

Parameter layout (one flat vector): W1 (H x I), b1 (H), W2 (H x H), b2 (H),
W3 (O x H), b3 (O), row-major.
"""
from __future__ import annotations

import math

import numpy as np

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The input is first rounded to float32, as the device holds it."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def _erf(z):
    return np.vectorize(math.erf, otypes=[np.float64])(z)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / _SQRT2))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


def param_count(n_in: int, n_hidden: int, n_out: int) -> int:
    return n_hidden * n_in + n_hidden + n_hidden * n_hidden + n_hidden + n_out * n_hidden + n_out


def unpack(params, n_in: int, n_hidden: int, n_out: int):
    p = np.asarray(params, dtype=np.float64)
    shapes = [(n_hidden, n_in), (n_hidden,), (n_hidden, n_hidden), (n_hidden,), (n_out, n_hidden),
              (n_out,)]
    out, o = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(p[o:o + size].reshape(s))
        o += size
    assert o == p.size
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in parts])


def _mm(a, b, rounded):
    """a @ b with both operands rounded to bfloat16 when ``rounded``."""
    if rounded:
        a, b = bf16(a), bf16(b)
    return a @ b


def forward(params, X, n_in, n_hidden, n_out, bf16_ops=True):
    """Returns (Y, cache) for inputs X (B x I).  With ``bf16_ops`` the
    parameters themselves are bfloat16 values (rounded here)."""
    W1, b1, W2, b2, W3, b3 = unpack(bf16(params) if bf16_ops else params, n_in, n_hidden, n_out)
    X = np.asarray(X, dtype=np.float64)
    z1 = _mm(X, W1.T, bf16_ops) + b1
    a1 = gelu(z1)
    z2 = _mm(a1, W2.T, bf16_ops) + b2
    a2 = gelu(z2)
    Y = _mm(a2, W3.T, bf16_ops) + b3
    return Y, (X, z1, a1, z2, a2)


def loss(Y, T):
    Y, T = np.asarray(Y, dtype=np.float64), np.asarray(T, dtype=np.float64)
    return 0.5 * np.mean((Y - T) ** 2)


def backward(params, X, T, n_in, n_hidden, n_out, bf16_ops=True):
    """Loss and its gradient with respect to the flat parameter vector."""
    W1, b1, W2, b2, W3, b3 = unpack(bf16(params) if bf16_ops else params, n_in, n_hidden, n_out)
    Y, (X, z1, a1, z2, a2) = forward(params, X, n_in, n_hidden, n_out, bf16_ops)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    dY = (Y - T) / (B * n_out)
    gW3 = _mm(dY.T, a2, bf16_ops)
    gb3 = dY.sum(axis=0)
    dz2 = _mm(dY, W3, bf16_ops) * gelu_grad(z2)
    gW2 = _mm(dz2.T, a1, bf16_ops)
    gb2 = dz2.sum(axis=0)
    dz1 = _mm(dz2, W2, bf16_ops) * gelu_grad(z1)
    gW1 = _mm(dz1.T, X, bf16_ops)
    gb1 = dz1.sum(axis=0)
    return loss(Y, T), pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (step counts from 1).  Returns (params, m, v)."""
    p, g = np.asarray(params, dtype=np.float64), np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
