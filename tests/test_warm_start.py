"""What the learned warm start gains over GN-MPPI from zero (chain16, N=50,
K=4096, float32).

The network is trained here, on the GPU, by the library's own kernels, on
(x0, U*) pairs produced by the solver from initial states drawn like the
instance's own; it is then judged on held-out initial states against plain
GN-MPPI started from zero, with C* per state taken from a longer GN-MPPI run
from zero (the solver is its own judge; the nonlinear chain has no closed-form
optimum).  The zero start is also the fallback: a proposal that costs more
than U = 0 is never used.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from paper_2512_04579_amd import _lib
from paper_2512_04579_amd.problem import DeviceProblem
from paper_2512_04579_amd.solver import GNMPPI
from paper_2512_04579_amd.warmstart import WarmStartNet, solve_pairs, start_controls

pytestmark = pytest.mark.gpu


def _gaps(w, dp, solver, graph, x0s, starts, cstar, iters):
    """Relative gaps of C(U_start) and of the cost after each iteration."""
    out = []
    for x0, U0, cs in zip(x0s, starts, cstar):
        solver.x0.copy_(torch.as_tensor(x0, dtype=torch.float32))
        solver.U.copy_(U0)
        c_start = torch.empty(1, dtype=torch.float32, device=dp.device)
        _lib.gnmppi_rollout(dp, solver.x0, solver.U, None, 0, None, None, None, c_start)
        graph.replay()
        costs = solver.info[:iters, 1].cpu().numpy()
        out.append(np.concatenate([[c_start.item()], costs]))
    out = np.array(out)
    return (out - cstar[:, None]) / np.abs(cstar[:, None])


def test_warm_start_beats_the_zero_start():
    w = wl.c2()
    p = w.problem
    X_train = wl.chain_initial_states(3072, seed=11)
    U_train, _, worst = solve_pairs(w, X_train, iters=4)
    assert (worst == 0).all()
    net = WarmStartNet(p.nx, p.n, seed=3)
    hist = net.fit(X_train, U_train, epochs=60, batch=256, lr=2e-3)
    assert hist[-1] < 0.05 * hist[0], hist

    X_test = wl.chain_initial_states(24, seed=12)
    Ustar, cstar, worst = solve_pairs(w, X_test, iters=10)
    assert (worst == 0).all()

    dp = DeviceProblem(p, "f32")
    iters = 2
    solver = GNMPPI(dp, w.x0, w.settings, seed=w.noise_seed + 50, max_iters=iters)
    graph = solver.capture(iters)
    zero_starts, warm_starts, chosen = [], [], []
    for x0 in X_test:
        x0d = dp.tensor(x0)
        U = torch.zeros(p.n, dtype=torch.float32, device=dp.device)
        info = start_controls(net, dp, x0d, U)
        chosen.append("network" if info[0].item() == 1.0 else "zero")
        warm_starts.append(U.clone())
        zero_starts.append(torch.zeros_like(U))
    g_zero = _gaps(w, dp, solver, graph, X_test, zero_starts, cstar, iters)
    g_warm = _gaps(w, dp, solver, graph, X_test, warm_starts, cstar, iters)
    med_zero, med_warm = np.median(g_zero, 0), np.median(g_warm, 0)
    print(f"\nnetwork start chosen for {chosen.count('network')} of {len(chosen)} held-out states")
    print("median relative gap   start      after 1 it  after 2 its")
    print(f"  zero start          {med_zero[0]:.3e}  {med_zero[1]:.3e}  {med_zero[2]:.3e}")
    print(f"  warm start          {med_warm[0]:.3e}  {med_warm[1]:.3e}  {med_warm[2]:.3e}")
    assert chosen.count("network") >= 0.9 * len(chosen)
    # the proposal alone is far closer to the optimum than U = 0 ...
    assert med_warm[0] < 0.01 * med_zero[0]
    # ... and one GN-MPPI iteration from it lands closer than one from zero
    assert med_warm[1] < med_zero[1]


def test_start_controls_falls_back_to_zero():
    """A proposal that costs more than U = 0 is not taken."""
    w = wl.c2()
    p = w.problem
    dp = DeviceProblem(p, "f32")
    net = WarmStartNet(p.nx, p.n, seed=0)
    with torch.no_grad():
        net.master.mul_(0.0)
        net.master[-p.n:] = 50.0   # b3: a huge constant control sequence
    net.params = net.master.to(torch.bfloat16)
    net._folded = None
    U = torch.full((p.n,), 7.0, dtype=torch.float32, device=dp.device)
    info = start_controls(net, dp, dp.tensor(w.x0), U)
    assert info[0].item() == 0.0 and info[2].item() == 1
    assert torch.count_nonzero(U).item() == 0
