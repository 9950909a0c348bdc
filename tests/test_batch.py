"""Batched GN-MPPI over uneven chain instances (one enqueue per iteration,
persistent launches per step and shape class).

Parity: every instance of a small uneven batch -- masses 3..16 (all three
lane-group classes), horizons 7..33 (several MFMA-tile and sweep classes),
K 64..512 -- after one iteration against the FP64 oracle fed the same Philox
stream (instance b uses key seed + b); a batch with one instance per shape
class the 1024-instance workload runs (contraction and G-sweep classes 3..10,
GGN-sweep classes 3..11, lane groups of 4, 8 and 16, K 512..4096) the same
way; after two iterations against the single-instance solver; graph replays
against eager iterations; every tuning against the default one.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl
from _parity import TOL, assert_parity, rel_err, rnd, round_problem
from oracle import ggn, jacobian, ocp, philox, solvers
from paper_2512_04579_amd import _lib
from paper_2512_04579_amd.batch import BatchGNMPPI, autotune
from paper_2512_04579_amd.problem import DeviceProblem
from paper_2512_04579_amd.solver import GNMPPI

# K = 100: a last k-step of 4 values (K % 32 == 4) in the batched contraction
SHAPES = [(3, 7, 64), (4, 12, 96), (5, 20, 128), (6, 10, 100), (8, 9, 256), (9, 33, 384),
          (16, 16, 512)]


def _instances():
    out = []
    for i, (M, N, K) in enumerate(SHAPES):
        prob, x0 = wl.chain_problem(n_masses=M, N=N, dt=0.05, seed=40 + i)
        out.append((prob, x0, K))
    return out


def _settings():
    return wl.SolverSettings(iters=3, K=0, sigma0=0.3, beta=0.9, sigma_min=1e-3, gamma=0.5,
                             n_alpha=16, contraction="bf16x3")


# rollout_mode 1: lane-group rollout storing the residuals, then the BF16x3
# contraction; 2: one lane per sample fused with the contraction
MODES = [1, 2]


@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_batch_first_iteration_matches_oracle(mode):
    inst = _instances()
    st = _settings()
    batch = BatchGNMPPI(inst, st, seed=11, tuning={"rollout_mode": mode})
    batch.step(0)
    torch.cuda.synchronize()
    status = batch.status.cpu().numpy()
    info = batch.info.cpu().numpy()
    assert (status == 0).all(), status
    for b, (p, x0, K) in enumerate(inst):
        rp = round_problem(p, "f32")
        noise = lambda it, s, K=K, p=p, b=b: rnd(philox.perturbations(p.n, K, s, 11 + b, it, "f32"), "f32")  # noqa: E731
        Uo, h = solvers.gn_mppi(rp, rnd(x0, "f32"), np.zeros(p.n), 1, noise, st.sigma0, beta=st.beta,
                                sigma_min=st.sigma_min)
        assert info[b, 0] == h.alpha[0], (b, info[b], h.alpha)
        assert_parity([info[b, 1]], [h.cost[0]], "f32", f"instance {b} cost")
        assert_parity(batch.controls(b).double().cpu().numpy(), Uo, "f32", f"instance {b} U")


# One instance per shape class of the 1024-instance workload (M in 4..16, N in
# 20..80, K in {512 .. 4096}): 16-column MFMA classes ceil(2N / 16) = 3..10 of
# the contraction, the J^T J tiles and the G sweep, GGN-sweep classes
# ceil((2N + 1) / 16) = 3..11, and lane groups of 4, 8 and 16 per sample.
C3_SHAPES = [(4, 20, 512), (5, 28, 1024), (9, 36, 2048), (16, 44, 4096), (4, 52, 1024),
             (5, 60, 2048), (9, 66, 4096), (16, 76, 2048), (12, 79, 512), (16, 80, 4096)]


@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_batch_every_c3_shape_class_matches_oracle(mode):
    inst = []
    for i, (M, N, K) in enumerate(C3_SHAPES):
        prob, x0 = wl.chain_problem(n_masses=M, N=N, dt=0.05, seed=70 + i)
        inst.append((prob, x0, K))
    classes = {(-(-p.n // 16), -(-(p.n + 1) // 16)) for p, _, _ in inst}
    assert {c for c, _ in classes} == set(range(3, 11)) and {h for _, h in classes} == set(range(3, 12))
    st = _settings()
    batch = BatchGNMPPI(inst, st, seed=31, tuning={"rollout_mode": mode})
    batch.step(0)
    torch.cuda.synchronize()
    status, info = batch.status.cpu().numpy(), batch.info.cpu().numpy()
    assert (status == 0).all(), status
    sig = st.sigma0  # iteration 0
    alphas = rnd(0.5 ** np.arange(st.n_alpha), "f32")
    for b, (p, x0, K) in enumerate(inst):
        rp, x0r = round_problem(p, "f32"), rnd(x0, "f32")
        W = rnd(philox.perturbations(p.n, K, sig, 31 + b, 0, "f32"), "f32")
        R, _ = ocp.rollout_batch(rp, x0r, np.zeros(p.n), W, nominal=True)
        d_ref = ggn.direction(jacobian.ls(R, W), R[:, 0])
        C_ref = ocp.cost_from_residual(ocp.residual(rp, x0r, d_ref[:, None] * alphas[None, :]))
        j = int(info[b, 2])
        # the device's step length is an argmin of the oracle's candidate costs
        assert 0 <= j < st.n_alpha and info[b, 0] == alphas[j], (b, info[b])
        assert C_ref[j] <= C_ref.min() * (1 + 10 * TOL["f32"]), (b, j, C_ref)
        assert_parity([info[b, 1]], [C_ref[j]], "f32", f"instance {b} {C3_SHAPES[b]} cost")
        assert_parity(batch.controls(b).double().cpu().numpy(), alphas[j] * d_ref, "f32",
                      f"instance {b} {C3_SHAPES[b]} U")


@pytest.mark.gpu
def test_fused_rollout_contraction_matches_the_unfused_path():
    # the same iteration through both mappings: S from the pair differences
    # contracted on chip against S from the stored residuals.  Both sum BF16x3
    # products (hi hi + hi lo + lo hi of bf16 splits, about 2^-17 relative per
    # product) of differently rounded operands in a different order, so each
    # is within the float32 bar of the oracle and they agree to that bar
    inst = _instances()
    for i, (M, N, K) in enumerate(C3_SHAPES[-3:]):
        prob, x0 = wl.chain_problem(n_masses=M, N=N, dt=0.05, seed=90 + i)
        inst.append((prob, x0, K))
    st = _settings()
    out = {}
    for mode in MODES:
        batch = BatchGNMPPI(inst, st, seed=13, tuning={"rollout_mode": mode})
        batch.step(0)
        torch.cuda.synchronize()
        assert (batch.status.cpu().numpy() == 0).all()
        out[mode] = (batch.U.cpu().numpy().astype(np.float64), batch.info.cpu().numpy())
    for b in range(len(inst)):
        sl = slice(int(batch.n_off[b]), int(batch.n_off[b + 1]))
        assert out[2][1][b, 0] == out[1][1][b, 0], (b, out[2][1][b], out[1][1][b])
        e = assert_parity(out[2][0][sl], out[1][0][sl], "f32", f"instance {b} U")
        print(f"instance {b} {batch.problems[b].n_masses, batch.problems[b].N, int(batch.K[b])}: "
              f"U fused vs unfused {e:.2e}")
        assert_parity([out[2][1][b, 1]], [out[1][1][b, 1]], "f32", f"instance {b} cost")


@pytest.mark.gpu
def test_batch_matches_the_single_instance_solver():
    inst = _instances()
    st = _settings()
    batch = BatchGNMPPI(inst, st, seed=21)
    for it in range(2):
        batch.step(it)
    torch.cuda.synchronize()
    for b, (p, x0, K) in enumerate(inst):
        s1 = wl.SolverSettings(iters=2, K=K, sigma0=st.sigma0, beta=st.beta, sigma_min=st.sigma_min,
                               gamma=st.gamma, n_alpha=st.n_alpha, contraction="bf16x3")
        single = GNMPPI(DeviceProblem(p, "f32"), x0, s1, seed=21 + b, max_iters=2)
        single.solve(2)
        torch.cuda.synchronize()
        costs, alphas, status = single.history(2)
        assert (status == 0).all()
        assert_parity([batch.info[b, 1].item()], [costs[1]], "f32", f"instance {b} cost")
        # the second step is small near the optimum; when the two solvers'
        # candidate costs are within rounding of each other they may pick
        # different step lengths, both valid, and then U differs by that
        # fraction of the step: U is compared when the step lengths agree
        print(f"instance {b}: alpha batch {batch.info[b, 0].item()} single {alphas[1]}; U rel diff "
              f"{rel_err(batch.controls(b).double().cpu().numpy(), single.U.double().cpu().numpy()):.2e}")
        if batch.info[b, 0].item() == alphas[1]:
            assert_parity(batch.controls(b).double().cpu().numpy(), single.U.double().cpu().numpy(),
                          "f32", f"instance {b} U")
        else:
            C_single = single.C_line.double().cpu().numpy()
            j = int(batch.info[b, 2].item())
            assert C_single[j] <= C_single.min() * (1 + 10 * TOL["f32"]), (b, j, C_single)


@pytest.mark.gpu
def test_batch_graph_replays_match_eager_iterations():
    inst = _instances()
    st = _settings()
    eager = BatchGNMPPI(inst, st, seed=5)
    for it in range(2):
        eager.step(it)
    torch.cuda.synchronize()
    U_ref, info_ref = eager.U.cpu().numpy(), eager.info.cpu().numpy()
    g = BatchGNMPPI(inst, st, seed=5)
    graph = g.capture(2)
    for rep in range(3):
        g.U.zero_()
        g.info.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.U.cpu().numpy(), U_ref, err_msg=f"replay {rep}")
        np.testing.assert_array_equal(g.info.cpu().numpy(), info_ref, err_msg=f"replay {rep}")


@pytest.mark.gpu
def test_batch_tunings_compute_the_same_iteration(tmp_path):
    inst = _instances()
    st = _settings()
    ref = BatchGNMPPI(inst, st, seed=8)
    ref.step(0)
    torch.cuda.synchronize()
    U_ref = ref.U.cpu().numpy()
    for tuning in ({"contract_ksplit": 1, "rollout_blocks_per_cu": 1, "rollout_mode": 1},
                   {"contract_ksplit": 4, "contract_blocks_per_cu": 4, "small_blocks_per_cu": 1,
                    "rollout_mode": 1},
                   {"rollout_mode": 2, "small_blocks_per_cu": 1}):
        b = BatchGNMPPI(inst, st, seed=8, tuning=tuning)
        b.step(0)
        torch.cuda.synchronize()
        assert_parity(b.U.cpu().numpy(), U_ref, "f32", str(tuning))
    b = BatchGNMPPI(inst, st, seed=8)
    entry = autotune(b, space=[{"rollout_mode": (2,)},
                               {"rollout_mode": (1,), "contract_ksplit": (1, 2),
                                "rollout_blocks_per_cu": (1, 2)}], reps=1,
                     cache=str(tmp_path / "tune.json"))
    assert entry["candidates"] == 5 and entry["tuning"] == b.tuning
    b.step(0)
    torch.cuda.synchronize()
    assert_parity(b.U.cpu().numpy(), U_ref, "f32", "autotuned")


def test_batch_rejects_invalid_instances():
    lib = _lib.load()
    shared = _lib.GnmppiProblem(model=_lib.MODEL_CHAIN, dtype=_lib.F32, nx=0, nu=0, N=0, n_masses=0,
                                dt=0.05, k_lin=1.0, k_cub=0.5, mass=1.0, q=None, r=None, x_ref=None)
    arr = (_lib.GnmppiBatchInstance * 2)()
    for a in arr:
        a.n_masses, a.N, a.K = 8, 20, 128
        a.x0 = a.q = a.r = a.x_ref = a.U = a.status = a.info = 0x1000
    st = _lib.GnmppiBatchSettings(seed=1, gamma=0.5, n_alpha=16, reserved=0, lm_lambda=0.0)
    tu = _lib.GnmppiBatchTuning()
    args = lambda: (ctypes.byref(shared), 2, arr, ctypes.byref(st), ctypes.byref(tu))  # noqa: E731
    ws = lib.gnmppi_batch_workspace(*args())
    assert ws > 0
    arr[1].K = 64  # K / 2 < n = 40: the antithetic pairs do not span the decisions
    assert lib.gnmppi_batch_workspace(*args()) == 0
    arr[1].K = 128
    arr[1].n_masses = 2
    assert lib.gnmppi_batch_workspace(*args()) == 0
    arr[1].n_masses = 8
    arr[1].N = 81
    assert lib.gnmppi_batch_workspace(*args()) == 0
    arr[1].N = 20
    st.n_alpha = 65
    assert lib.gnmppi_batch_workspace(*args()) == 0
    st.n_alpha = 16
    assert lib.gnmppi_batch_prepare(*args(), 0x1008, ws) == _lib.EINVAL          # misaligned
    assert lib.gnmppi_batch_prepare(*args(), 0x1000, ws - 1) == _lib.ENOSPACE
    assert lib.gnmppi_batch_iteration(*args(), 0x1000, ws, 0, 0.0, None) == _lib.EINVAL  # sigma
    shared.dtype = _lib.F64
    assert lib.gnmppi_batch_workspace(*args()) == 0
