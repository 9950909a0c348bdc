"""GPU parity of the warm-start network kernels against the FP64 oracle
(oracle/mlp.py) on identical bfloat16 parameters and float32 inputs.

Tolerance, derived from the arithmetic: both sides round every product
operand to bfloat16 and then sum exactly representable products, the device
in float32 (relative error <= K 2^-24 ~ 1.5e-5 for K <= 256, ~1e-6 typical).
An intermediate (a hidden activation, dY) that the device holds in float32
and the oracle in float64 can round to a neighbouring bfloat16 value when it
sits next to a rounding boundary; such flips hit a fraction ~1e-4 of the
elements, each by 2^-8 relative, i.e. ~1e-4 normwise at most.  Hence 1e-4
normwise for the forward pass, 5e-4 for the gradients (which pass through two
more rounded operands), and 1e-6 of each array's scale for the Adam update.

Shapes: the warm-start network (64 -> 256 -> 256 -> 100) at a batch of 1024,
and a ragged one (37 -> 70 -> 70 -> 23, batch 133) whose every dimension
leaves a partial MFMA tile.
"""
import numpy as np
import pytest
import torch

from _parity import rel_err
from oracle import mlp
from paper_2512_04579_amd import _lib

pytestmark = pytest.mark.gpu

SHAPES = [(64, 256, 100, 1024), (37, 70, 23, 133)]


def _net(I, H, O, B, seed):
    rng = np.random.default_rng(seed)
    P = mlp.param_count(I, H, O)
    scale = np.concatenate([np.full(H * I, 1 / np.sqrt(I)), np.full(H, 0.1), np.full(H * H, 1 / np.sqrt(H)),
                            np.full(H, 0.1), np.full(O * H, 1 / np.sqrt(H)), np.full(O, 0.1)])
    p = mlp.bf16(rng.standard_normal(P) * scale)
    X = rng.uniform(-1, 1, (B, I)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((B, O)).astype(np.float32).astype(np.float64)
    dev = torch.device("cuda")
    pd = torch.tensor(p, dtype=torch.float32, device=dev).to(torch.bfloat16)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    Td = torch.tensor(T, dtype=torch.float32, device=dev)
    work = torch.empty(_lib.gnmppi_mlp_workspace(I, H, O, B), dtype=torch.uint8, device=dev)
    return p, X, T, pd, Xd, Td, work


@pytest.mark.parametrize("I,H,O,B", SHAPES)
def test_mlp_forward_matches_oracle(I, H, O, B):
    p, X, T, pd, Xd, Td, work = _net(I, H, O, B, 1)
    assert _lib.gnmppi_mlp_param_count(I, H, O) == p.size
    Y = torch.empty(B, O, dtype=torch.float32, device="cuda")
    _lib.gnmppi_mlp_forward((I, H, O), pd, Xd, Y, work)
    torch.cuda.synchronize()
    ref, _ = mlp.forward(p, X, I, H, O, bf16_ops=True)
    e = rel_err(Y.double().cpu().numpy(), ref)
    print(f"forward {I}-{H}-{O} B={B}: {e:.2e}")
    assert e < 1e-4


@pytest.mark.parametrize("I,H,O,B", SHAPES)
def test_mlp_backward_matches_oracle(I, H, O, B):
    p, X, T, pd, Xd, Td, work = _net(I, H, O, B, 2)
    grad = torch.full((p.size,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    _lib.gnmppi_mlp_backward((I, H, O), pd, Xd, Td, loss, grad, work)
    torch.cuda.synchronize()
    Lref, gref = mlp.backward(p, X, T, I, H, O, bf16_ops=True)
    assert abs(loss.item() - Lref) / Lref < 1e-5
    g = grad.double().cpu().numpy()
    assert np.isfinite(g).all()
    for name, (a, b) in zip(["W1", "b1", "W2", "b2", "W3", "b3"],
                            zip(mlp.unpack(g, I, H, O), mlp.unpack(gref, I, H, O))):
        e = rel_err(a, b)
        print(f"grad {name} {I}-{H}-{O} B={B}: {e:.2e}")
        assert e < 5e-4, name


def test_mlp_adam_step_matches_oracle():
    rng = np.random.default_rng(4)
    P = 100003
    master = rng.standard_normal(P).astype(np.float32)
    g = (rng.standard_normal(P) * 1e-2).astype(np.float32)
    m = (rng.standard_normal(P) * 1e-3).astype(np.float32)
    v = (rng.uniform(0, 1e-4, P)).astype(np.float32)
    dev = torch.device("cuda")
    md, gd, mmd, vd = (torch.tensor(a, device=dev) for a in (master, g, m, v))
    pb = torch.empty(P, dtype=torch.bfloat16, device=dev)
    _lib.gnmppi_mlp_adam(md, pb, gd, mmd, vd, 1e-3, 7)
    torch.cuda.synchronize()
    ref_p, ref_m, ref_v = mlp.adam(master, g, m, v, 7, 1e-3)
    # float32 arithmetic with beta1 = 0.9 and 1 - beta1 rounded to float32:
    # ~1e-7 of each array's scale (the moments cancel, so no relative bound)
    for got, ref in ((md, ref_p), (mmd, ref_m), (vd, ref_v)):
        np.testing.assert_allclose(got.double().cpu().numpy(), ref, rtol=0,
                                   atol=1e-6 * np.abs(ref).max())
    np.testing.assert_array_equal(pb.double().cpu().numpy(), mlp.bf16(md.double().cpu().numpy()))


def test_mlp_training_reduces_the_loss():
    """A few hundred Adam steps of the device kernels fit a smooth target."""
    I, H, O, B = 8, 64, 4, 256
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (B, I))
    T = np.stack([np.sin(X[:, 0] + X[:, 1]), X[:, 2] * X[:, 3], np.cos(X[:, 4]), X[:, 5] ** 2], 1)
    dev = torch.device("cuda")
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    Td = torch.tensor(T, dtype=torch.float32, device=dev)
    P = _lib.gnmppi_mlp_param_count(I, H, O)
    init = rng.standard_normal(P) * 0.2
    master = torch.tensor(init, dtype=torch.float32, device=dev)
    params = master.to(torch.bfloat16)
    m, v = torch.zeros_like(master), torch.zeros_like(master)
    grad = torch.zeros_like(master)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    work = torch.empty(_lib.gnmppi_mlp_workspace(I, H, O, B), dtype=torch.uint8, device=dev)
    losses = []
    for step in range(1, 401):
        _lib.gnmppi_mlp_backward((I, H, O), params, Xd, Td, loss, grad, work)
        _lib.gnmppi_mlp_adam(master, params, grad, m, v, 3e-3, step)
        if step in (1, 400):
            losses.append(loss.item())
    assert losses[1] < 0.1 * losses[0], losses
