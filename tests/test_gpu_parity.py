"""GPU parity: each C-ABI call against the FP64 oracle on identical seeded,
dtype-rounded inputs (float32 <= 1e-4, float64 <= 1e-10 normwise relative).

Cases span several tiles with ragged tails, the full c2 shapes (chain16,
N=50, K=4096, the launch configuration the benchmark times), the limits
(n = 192, L = 1 and 64, K = 0 and 1, a single-mass chain) and the
degenerate inputs (non-finite costs, rank-deficient perturbations, a
singular normal matrix).
"""
import json
import os
import zlib

import numpy as np
import pytest
import torch

import workloads as wl
from _parity import TOL, assert_parity, device, host, padded, rel_err, rnd, round_problem, to_dev
from oracle import dynamics, ggn, jacobian, lqr, mppi, ocp, philox, sigma_points, solvers
from paper_2512_04579_amd import _lib
from paper_2512_04579_amd.problem import DeviceProblem
from paper_2512_04579_amd.solver import SCHEDULES, GNMPPI, PlainMPPI, make_solver

pytestmark = pytest.mark.gpu


def _sync():
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# a1: sampler
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,n,K,anti", [("f32", 37, 300, True), ("f64", 37, 300, True),
                                             ("f32", 100, 4096, True), ("f32", 5, 77, False),
                                             ("f64", 3, 1, False)])
def test_sampler_matches_philox_definition(dtype, n, K, anti):
    dev = device()
    W = padded(np.zeros((n, K)), dtype)
    _lib.gnmppi_sample(W, 0.3, seed=0x1234_5678_9ABC, stream_id=7, antithetic=anti, K=K)
    _sync()
    ref = philox.perturbations(n, K, 0.3, seed=0x1234_5678_9ABC, stream=7, dtype=dtype, antithetic=anti)
    got = host(W)
    tol = 2e-6 if dtype == "f32" else 1e-13
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol)
    if anti:
        np.testing.assert_array_equal(got[:, K // 2:], -got[:, :K // 2])


def test_sigma_points_match_method_e_set():
    n = 40
    W = padded(np.zeros((n, 2 * n)), "f64")
    _lib.gnmppi_sigma_points(W, 0.25)
    _sync()
    np.testing.assert_allclose(host(W), sigma_points.symmetric_set(n, 0.25), rtol=1e-15, atol=0)


# ---------------------------------------------------------------------------
# a2: rollout
# ---------------------------------------------------------------------------

def _rollout_case(name):
    if name == "c1":
        w = wl.c1()
        return w.problem, w.x0, "f64", 256, True
    if name == "c2":
        w = wl.c2()
        return w.problem, w.x0, "f32", 4096, True
    if name == "di_axis_N50_ragged":
        p = wl.double_integrator_problem(axes=1, N=50)
        return p, np.array([0.7, -0.3]), "f64", 301, False
    if name == "chain3_f32_ragged":
        p, x0 = wl.chain_problem(n_masses=3, N=6, seed=3)
        return p, x0, "f32", 300, True
    if name == "chain5_f64_padding_lanes":
        p, x0 = wl.chain_problem(n_masses=5, N=7, seed=4)
        return p, x0, "f64", 257, False
    if name == "chain1_f32":
        p, x0 = wl.chain_problem(n_masses=1, N=4, seed=5)
        return p, x0, "f32", 65, False
    if name == "chain16_f64":
        p, x0 = wl.chain_problem(n_masses=16, N=12, seed=6)
        return p, x0, "f64", 128, True
    raise KeyError(name)


@pytest.mark.parametrize("name", ["c1", "c2", "di_axis_N50_ragged", "chain3_f32_ragged",
                                  "chain5_f64_padding_lanes", "chain1_f32", "chain16_f64"])
def test_rollout_matches_oracle(name):
    prob, x0, dtype, K, anti = _rollout_case(name)
    dev = device()
    rp = round_problem(prob, dtype)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    U = rnd(0.2 * rng.standard_normal(prob.n), dtype)
    W = rnd(wl.gaussian_perturbations(prob.n, K, 0.3, 11, antithetic=anti), dtype)
    x0r = rnd(x0, dtype)
    dp = DeviceProblem(prob, dtype)
    Wd, Rd = padded(W, dtype), padded(np.zeros((prob.m, K)), dtype)
    Cd = to_dev(np.zeros(K), dtype)
    r0d, c0d = to_dev(np.zeros(prob.m), dtype), to_dev(np.zeros(1), dtype)
    x0d, Ud = to_dev(x0r, dtype), to_dev(U, dtype)
    _lib.gnmppi_rollout(dp, x0d, Ud, Wd, K, Rd, Cd, r0d, c0d)
    # costs-only launch must reproduce the stored-run costs bit for bit
    C2 = to_dev(np.zeros(K), dtype)
    _lib.gnmppi_rollout(dp, x0d, Ud, Wd, K, None, C2)
    _sync()
    R_ref, C_ref = ocp.rollout_batch(rp, x0r, U, W, nominal=True)
    assert_parity(host(Rd), R_ref[:, 1:], dtype, "R")
    assert_parity(host(Cd), C_ref[1:], dtype, "C")
    assert_parity(host(r0d), R_ref[:, 0], dtype, "r0")
    assert_parity(host(c0d), C_ref[:1], dtype, "c0")
    np.testing.assert_array_equal(host(C2), host(Cd))
    # residuals-only launch (no C, as the GN-MPPI step calls it): the same R,
    # r0 and c0 bit for bit
    R3 = padded(np.zeros((prob.m, K)), dtype)
    r03, c03 = to_dev(np.zeros(prob.m), dtype), to_dev(np.zeros(1), dtype)
    _lib.gnmppi_rollout(dp, x0d, Ud, Wd, K, R3, None, r03, c03)
    _sync()
    np.testing.assert_array_equal(host(R3), host(Rd))
    np.testing.assert_array_equal(host(r03), host(r0d))
    np.testing.assert_array_equal(host(c03), host(c0d))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_rollout_nominal_only_and_single_sample(dtype):
    prob, x0 = wl.chain_problem(n_masses=4, N=9, seed=8)
    rp = round_problem(prob, dtype)
    dp = DeviceProblem(prob, dtype)
    U = rnd(np.linspace(-0.5, 0.5, prob.n), dtype)
    x0r = rnd(x0, dtype)
    c0 = to_dev(np.zeros(1), dtype)
    r0 = to_dev(np.zeros(prob.m), dtype)
    _lib.gnmppi_rollout(dp, to_dev(x0r, dtype), to_dev(U, dtype), None, 0, None, None, r0, c0)
    W1 = rnd(0.1 * np.ones((prob.n, 1)), dtype)
    C1 = to_dev(np.zeros(1), dtype)
    _lib.gnmppi_rollout(dp, to_dev(x0r, dtype), to_dev(U, dtype), padded(W1, dtype), 1, None, C1)
    _sync()
    assert_parity(host(r0), ocp.residual(rp, x0r, U), dtype, "r0")
    assert_parity(host(c0), [ocp.cost(rp, x0r, U)], dtype, "c0")
    assert_parity(host(C1), [ocp.cost(rp, x0r, U + W1[:, 0])], dtype, "C1")


@pytest.mark.parametrize("K", [61, 65, 4090])
def test_rollout_residual_layouts_agree(K):
    # R with an odd leading dimension takes the scalar residual stores, the
    # padded R the 4-sample vector stores; both, and the ragged last chunk
    # left of the nominal column, must give the same bits (and c0 the same
    # sum of the staged nominal rows)
    prob, x0 = wl.chain_problem(n_masses=16, N=9, seed=12)
    dp = DeviceProblem(prob, "f32")
    rng = np.random.default_rng(K)
    U = rnd(0.2 * rng.standard_normal(prob.n), "f32")
    W = rnd(0.3 * rng.standard_normal((prob.n, K)), "f32")
    x0d, Ud, Wd = to_dev(rnd(x0, "f32"), "f32"), to_dev(U, "f32"), padded(W, "f32")
    outs = []
    for R, aligned in ((padded(np.zeros((prob.m, K)), "f32"), True),
                       (torch.zeros(prob.m, K + 1, dtype=torch.float32, device=device())[:, :K],
                        False)):
        assert (R.stride(0) % 4 == 0) == aligned
        r0, c0 = to_dev(np.zeros(prob.m), "f32"), to_dev(np.zeros(1), "f32")
        _lib.gnmppi_rollout(dp, x0d, Ud, Wd, K, R, None, r0, c0)
        _sync()
        outs.append((host(R), host(r0), host(c0)))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)
    rp = round_problem(prob, "f32")
    cols = [0, K // 2, K - 1]
    R_ref = np.stack([ocp.residual(rp, rnd(x0, "f32"), U + W[:, c]) for c in cols], axis=1)
    assert_parity(outs[0][0][:, cols], R_ref, "f32", "R sampled columns")
    assert_parity(outs[0][2], [ocp.cost(rp, rnd(x0, "f32"), U)], "f32", "c0")


def _solver(dp, w, schedule, **kw):
    return make_solver(dp, w.x0, w.settings, schedule, **kw)


@pytest.mark.parametrize("schedule", ["ahead", "prefetch", "same"])
def test_eager_steps_with_a_side_stream_match_one_stream(schedule):
    w = wl.c2()
    dp = DeviceProblem(w.problem, w.dtype)
    ref = _solver(dp, w, "formed", seed=9, max_iters=3)
    two = _solver(dp, w, schedule, seed=9, max_iters=3)
    for it in range(3):
        ref.step(it)
        two.step(it, ahead=it + 1 < 3)
    _sync()
    np.testing.assert_array_equal(host(two.U), host(ref.U))
    np.testing.assert_array_equal(host(two.info), host(ref.info))
    assert (two.history(3)[2] == 0).all()


@pytest.mark.parametrize("name,outputs", [("c2", "R"), ("c1", "R"), ("chain3_f32_ragged", "R"),
                                          ("chain5_f64_padding_lanes", "R"), ("chain1_f32", "R"),
                                          ("chain16_f64", "R"), ("c2", "C"), ("c2", "RC")])
def test_sample_rollout_equals_the_sampler_then_the_rollout(name, outputs):
    # one launch that draws W itself (chain, residuals wanted) or the two
    # calls in a row (double integrator, costs only): bit for bit the same W,
    # R, r0, c0 and C as gnmppi_sample followed by gnmppi_rollout
    prob, x0, dtype, K, anti = _rollout_case(name)
    dp = DeviceProblem(prob, dtype)
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    Ud = to_dev(rnd(0.2 * rng.standard_normal(prob.n), dtype), dtype)
    x0d = to_dev(rnd(x0, dtype), dtype)
    seed, sid, sigma = 0x5EED_0000_1234, 17, 0.3
    outs = []
    for fused in (False, True):
        Wd = padded(np.full((prob.n, K), 9.0), dtype, ld=K + 3)
        R = padded(np.zeros((prob.m, K)), dtype) if "R" in outputs else None
        C = to_dev(np.zeros(K), dtype) if "C" in outputs else None
        r0 = to_dev(np.zeros(prob.m), dtype) if "R" in outputs else None
        c0 = to_dev(np.zeros(1), dtype)
        if fused:
            _lib.gnmppi_sample_rollout(dp, x0d, Ud, Wd, sigma, seed, sid, K, antithetic=anti, R=R,
                                       C=C, r0=r0, c0=c0)
        else:
            _lib.gnmppi_sample(Wd, sigma, seed, sid, antithetic=anti, K=K)
            _lib.gnmppi_rollout(dp, x0d, Ud, Wd, K, R, C, r0, c0)
        _sync()
        outs.append([host(t) for t in (Wd, R, C, r0, c0) if t is not None])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(b, a)
    ref = philox.perturbations(prob.n, K, sigma, seed=seed, stream=sid, dtype=dtype, antithetic=anti)
    np.testing.assert_allclose(outs[1][0], ref, rtol=2e-6 if dtype == "f32" else 1e-13,
                               atol=2e-6 if dtype == "f32" else 1e-13)


def test_chain_rest_pose_is_a_fixed_point_on_device():
    prob, _ = wl.chain_problem(n_masses=16, N=50, seed=2)
    dp = DeviceProblem(prob, "f64")
    c0 = to_dev(np.ones(1), "f64")
    r0 = to_dev(np.ones(prob.m), "f64")
    _lib.gnmppi_rollout(dp, to_dev(prob.x_ref, "f64"), to_dev(np.zeros(prob.n), "f64"), None, 0,
                        None, None, r0, c0)
    _sync()
    assert np.abs(host(r0)).max() < 1e-13
    assert host(c0)[0] < 1e-25


# ---------------------------------------------------------------------------
# a3: MPPI update
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,n,K", [("f32", 37, 1000), ("f64", 37, 1000), ("f32", 100, 4096),
                                       ("f64", 40, 256), ("f32", 1, 1), ("f32", 3, 16384)])
def test_mppi_update_matches_oracle(dtype, n, K):
    rng = np.random.default_rng(n + K)
    W = rnd(rng.standard_normal((n, K)), dtype)
    C = rnd(rng.uniform(10.0, 14.0, K), dtype)
    if K > 8:
        C[3], C[5], C[7] = np.nan, np.inf, -np.inf
    U = rnd(rng.standard_normal(n), dtype)
    lam = 0.3
    Ud = to_dev(U, dtype)
    wd = to_dev(np.zeros(K), dtype)
    st = torch.full((1,), 99, dtype=torch.int32, device=device())
    _lib.gnmppi_mppi_update(to_dev(C, dtype), padded(W, dtype), lam, Ud, wd, st)
    _sync()
    assert int(st.item()) == _lib.OK
    assert_parity(host(Ud) - U, mppi.step(W, C, lam), dtype, "dU")
    assert_parity(host(wd), mppi.weights(C, lam), dtype, "weights")


def test_mppi_update_all_nonfinite_leaves_U():
    U = np.arange(5.0)
    Ud = to_dev(U, "f32")
    st = torch.zeros(1, dtype=torch.int32, device=device())
    C = np.array([np.nan, np.inf, np.nan, -np.inf])
    _lib.gnmppi_mppi_update(to_dev(C, "f32"), padded(np.ones((5, 4)), "f32"), 1.0, Ud, None, st)
    _sync()
    assert int(st.item()) == _lib.ENONFINITE
    np.testing.assert_array_equal(host(Ud), U)


# ---------------------------------------------------------------------------
# a4: Jacobian reconstruction
# ---------------------------------------------------------------------------

def _jacobian_inputs(case):
    if case == "c1":
        w = wl.c1()
        prob, x0, dtype, K, anti, sigma = w.problem, w.x0, "f64", 256, True, 0.5
    elif case == "c2":
        w = wl.c2()
        prob, x0, dtype, K, anti, sigma = w.problem, w.x0, "f32", 4096, True, 0.3
    elif case == "chain_f64_ragged":
        prob, x0 = wl.chain_problem(n_masses=3, N=5, seed=1)
        dtype, K, anti, sigma = "f64", 100, False, 0.2
    elif case == "chain_f32_ragged":
        prob, x0 = wl.chain_problem(n_masses=6, N=9, seed=2)
        dtype, K, anti, sigma = "f32", 333, False, 0.3
    else:
        raise KeyError(case)
    rp = round_problem(prob, dtype)
    U = rnd(0.1 * np.random.default_rng(3).standard_normal(prob.n), dtype)
    W = rnd(wl.gaussian_perturbations(prob.n, K, sigma, 21, antithetic=anti), dtype)
    R, _ = ocp.rollout_batch(rp, rnd(x0, dtype), U, W, nominal=True)
    R = rnd(R, dtype)  # the device receives the residuals in its own precision
    return prob, dtype, K, sigma, R, W


def _run_jacobian(R, W, dtype, method=_lib.JAC_LS, sigma2=0.0, ldw=None, ldr=None):
    m, K = R.shape[0], W.shape[1]
    n = W.shape[0]
    Rd = padded(R[:, 1:], dtype, ld=ldr)
    Wd = padded(W, dtype, ld=ldw)
    r0d = to_dev(R[:, 0], dtype)
    J = to_dev(np.zeros((m, n)), dtype)
    code = _lib.F32 if dtype == "f32" else _lib.F64
    work = torch.empty(_lib.gnmppi_jacobian_workspace(code, m, n, K), dtype=torch.uint8, device=device())
    st = torch.full((1,), 99, dtype=torch.int32, device=device())
    _lib.gnmppi_reconstruct_jacobian(Rd, r0d, Wd, J, work, method, sigma2, st, K)
    _sync()
    return host(J), int(st.item())


@pytest.mark.parametrize("case", ["c1", "c2", "chain_f64_ragged", "chain_f32_ragged"])
def test_jacobian_ls_matches_oracle(case):
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    J, st = _run_jacobian(R, W, dtype)
    assert st == _lib.OK
    assert_parity(J, jacobian.ls(R, W), dtype, "J (LS)")


@pytest.mark.parametrize("case", ["c1", "chain_f32_ragged"])
def test_jacobian_mc_matches_oracle(case):
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    J, st = _run_jacobian(R, W, dtype, _lib.JAC_MC, sigma * sigma)
    assert st == _lib.OK
    assert_parity(J, jacobian.mc(R, W, sigma * sigma), dtype, "J (MC)")


@pytest.mark.parametrize("case", ["c1", "c2", "chain_f32_ragged"])
def test_jacobian_with_gram_factored_separately(case):
    # gnmppi_perturbation_gram (W only) then GRAM_READY: same J as the oracle
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    m, n = R.shape[0], W.shape[0]
    Rd, Wd, r0d = padded(R[:, 1:], dtype), padded(W, dtype), to_dev(R[:, 0], dtype)
    J = to_dev(np.zeros((m, n)), dtype)
    code = _lib.F32 if dtype == "f32" else _lib.F64
    work = torch.empty(_lib.gnmppi_jacobian_workspace(code, m, n, K), dtype=torch.uint8, device=device())
    st = torch.full((2,), 99, dtype=torch.int32, device=device())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _lib.gnmppi_perturbation_gram(Wd, work, m, st[1:2], K)
    torch.cuda.current_stream().wait_stream(side)
    _lib.gnmppi_reconstruct_jacobian(Rd, r0d, Wd, J, work, _lib.JAC_LS | _lib.JAC_GRAM_READY, 0.0,
                                     st[0:1], K)
    _sync()
    assert host(st).tolist() == [0, 0]
    assert_parity(host(J), jacobian.ls(R, W), dtype, "J (gram on a side stream)")


@pytest.mark.parametrize("case", ["c2", "chain_f32_ragged"])
@pytest.mark.parametrize("contraction", [0, _lib.JAC_BF16X3])
def test_jacobian_in_two_phases_matches_one_call(case, contraction):
    # S_ONLY on the main stream while the gram runs on a side stream, then
    # APPLY_ONLY after the join: bit-identical to one GRAM_READY call
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    if dtype != "f32" and contraction:
        pytest.skip("BF16 contractions are F32 only")
    m, n = R.shape[0], W.shape[0]
    Rd, Wd, r0d = padded(R[:, 1:], dtype), padded(W, dtype), to_dev(R[:, 0], dtype)
    code = _lib.F32 if dtype == "f32" else _lib.F64
    nbytes = _lib.gnmppi_jacobian_workspace(code, m, n, K)
    method = _lib.JAC_LS | _lib.JAC_GRAM_READY | contraction
    out = []
    for split in (False, True):
        work = torch.empty(nbytes, dtype=torch.uint8, device=device())
        J = to_dev(np.zeros((m, n)), dtype)
        st = torch.full((2,), 99, dtype=torch.int32, device=device())
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _lib.gnmppi_perturbation_gram(Wd, work, m, st[1:2], K)
        if split:
            _lib.gnmppi_reconstruct_jacobian(Rd, r0d, Wd, J, work, method | _lib.JAC_S_ONLY, 0.0,
                                             st[0:1], K)
            torch.cuda.current_stream().wait_stream(side)
            _sync()
            assert host(st)[0] == 99  # S_ONLY writes no status
            _lib.gnmppi_reconstruct_jacobian(Rd, r0d, Wd, J, work, method | _lib.JAC_APPLY_ONLY, 0.0,
                                             st[0:1], K)
        else:
            torch.cuda.current_stream().wait_stream(side)
            _lib.gnmppi_reconstruct_jacobian(Rd, r0d, Wd, J, work, method, 0.0, st[0:1], K)
        _sync()
        assert host(st).tolist() == [0, 0]
        out.append(host(J))
    np.testing.assert_array_equal(out[1], out[0])
    assert_parity(out[1], jacobian.ls(R, W), dtype, "J (two phases)", tol=1e-3 if contraction else None)


def test_perturbation_gram_reports_rank_deficiency():
    rng = np.random.default_rng(6)
    n, K = 12, 10
    Wd = padded(rng.standard_normal((n, K)), "f64")
    work = torch.empty(_lib.gnmppi_jacobian_workspace(_lib.F64, 30, n, K), dtype=torch.uint8, device=device())
    st = torch.full((1,), 99, dtype=torch.int32, device=device())
    _lib.gnmppi_perturbation_gram(Wd, work, 30, st, K)
    _sync()
    assert int(st.item()) == _lib.ERANK


@pytest.mark.parametrize("case", ["c2", "chain_f32_ragged"])
@pytest.mark.parametrize("method", ["ls", "mc"])
def test_jacobian_bf16x3_split_keeps_fp32_accuracy(case, method):
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    code = (_lib.JAC_LS if method == "ls" else _lib.JAC_MC) | _lib.JAC_BF16X3
    J, st = _run_jacobian(R, W, dtype, code, sigma * sigma)
    assert st == _lib.OK
    ref = jacobian.ls(R, W) if method == "ls" else jacobian.mc(R, W, sigma * sigma)
    e = assert_parity(J, ref, "f32", "J (bf16x3)")
    assert e < 2e-5, e


def _linear_residuals(m, n, K, seed):
    # residual columns exactly linear in the perturbations, R[:, 1 + s] = r0 + A W[:, s]
    rng = np.random.default_rng(seed)
    W = rnd(0.3 * rng.standard_normal((n, K)), "f32")
    A = rng.standard_normal((m, n))
    r0 = rng.standard_normal(m)
    return rnd(np.concatenate([r0[:, None], r0[:, None] + A @ W], axis=1), "f32"), W


@pytest.mark.parametrize("n,K", [(5, 8), (5, 40), (37, 904), (37, 1000), (37, 4104)])
def test_bf16x3_contraction_with_a_ragged_last_step(n, K):
    # K % 8 == 0 takes the 16-byte load path; K % 32 != 0 leaves a last k-step
    # with fewer than 32 values, whose missing groups must read inside the row
    # (tight rows: the last row ends the allocation) and contribute zeros
    R, W = _linear_residuals(300, n, K, seed=K)
    code = _lib.JAC_LS | _lib.JAC_BF16X3
    J, st = _run_jacobian(R, W, "f32", code, ldw=K, ldr=K)
    assert st == _lib.OK
    assert_parity(J, jacobian.ls(R, W), "f32", f"J (bf16x3, K={K}, tight rows)")
    dU, st2 = _run_direction(R, W, "f32", code)
    assert st2 == [0, 0]
    assert_parity(dU, ggn.direction(jacobian.ls(R, W), R[:, 0], 0.0), "f32",
                  f"dU (bf16x3, K={K}, NaN past K in every row)")


def test_jacobian_bf16_precision_split_error_is_bounded():
    # plain BF16 operands: the error is the precision split's, reported, not FP32 parity
    prob, dtype, K, sigma, R, W = _jacobian_inputs("c2")
    J, st = _run_jacobian(R, W, dtype, _lib.JAC_LS | _lib.JAC_BF16)
    assert st == _lib.OK
    e = rel_err(J, jacobian.ls(R, W))
    print(f"BF16 precision split: J normwise relative error vs FP64 oracle {e:.3e}")
    assert 1e-5 < e < 3e-3, e


def test_jacobian_unaligned_leading_dimensions_take_the_scalar_path():
    prob, dtype, K, sigma, R, W = _jacobian_inputs("chain_f64_ragged")
    J, st = _run_jacobian(R, W, dtype, ldw=K + 1, ldr=K + 3)
    assert st == _lib.OK
    assert_parity(J, jacobian.ls(R, W), dtype, "J (unaligned)")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_jacobian_at_the_largest_supported_n(dtype):
    rng = np.random.default_rng(4)
    n, m, K = 192, 70, 512
    W = rnd(rng.standard_normal((n, K)), dtype)
    A = rng.standard_normal((m, n))
    r0 = rng.standard_normal(m)
    R = rnd(np.concatenate([r0[:, None], r0[:, None] + A @ W], axis=1), dtype)
    J, st = _run_jacobian(R, W, dtype)
    assert st == _lib.OK
    assert_parity(J, jacobian.ls(R, W), dtype, "J (n=192)")


def test_jacobian_reports_rank_deficient_perturbations():
    rng = np.random.default_rng(5)
    n, K = 12, 10
    W = rng.standard_normal((n, K))
    R = rng.standard_normal((30, K + 1))
    _, st = _run_jacobian(R, W, "f64")
    assert st == _lib.ERANK


# ---------------------------------------------------------------------------
# a5: GGN step
# ---------------------------------------------------------------------------

def _run_ggn(J, r0, lam, dtype, inc=1):
    m, n = J.shape
    Jd = to_dev(J, dtype)
    r0_full = np.zeros(m * inc)
    r0_full[::inc] = r0
    r0d = to_dev(r0_full, dtype)
    dU = to_dev(np.full(n, 7.0), dtype)
    code = _lib.F32 if dtype == "f32" else _lib.F64
    work = torch.empty(_lib.gnmppi_ggn_workspace(code, m, n), dtype=torch.uint8, device=device())
    st = torch.full((1,), 99, dtype=torch.int32, device=device())
    _lib.gnmppi_ggn_step(Jd, r0d, lam, dU, work, st, inc_r0=inc)
    _sync()
    return host(dU), int(st.item())


@pytest.mark.parametrize("dtype,m,n,lam,inc", [("f64", 120, 40, 0.0, 1), ("f32", 120, 40, 0.0, 1),
                                               ("f64", 300, 37, 0.5, 3), ("f32", 3300, 100, 0.0, 1),
                                               ("f64", 200, 192, 1e-3, 1), ("f32", 65, 1, 0.0, 2)])
def test_ggn_step_matches_oracle(dtype, m, n, lam, inc):
    rng = np.random.default_rng(m + n)
    J = rnd(rng.standard_normal((m, n)) + 0.3, dtype)
    r0 = rnd(rng.standard_normal(m), dtype)
    dU, st = _run_ggn(J, r0, lam, dtype, inc)
    assert st == _lib.OK
    assert_parity(dU, ggn.direction(J, r0, lam), dtype, "dU")


def test_ggn_step_on_the_c2_jacobian():
    prob, dtype, K, sigma, R, W = _jacobian_inputs("c2")
    J = rnd(jacobian.ls(R, W), dtype)
    dU, st = _run_ggn(J, R[:, 0], 0.0, dtype)
    assert st == _lib.OK
    assert_parity(dU, ggn.direction(J, R[:, 0]), dtype, "dU (c2)")


def test_ggn_step_reports_singular_normal_matrix():
    dU, st = _run_ggn(np.zeros((20, 6)), np.ones(20), 0.0, "f64")
    assert st == _lib.ENOTPD
    np.testing.assert_array_equal(dU, np.zeros(6))


@pytest.mark.parametrize("dup,src", [(17, 16), (25, 3), (26, 3), (39, 38), (32, 0)])
def test_ggn_step_detects_a_late_zero_pivot(dup, src):
    # column dup repeats column src: the Schur complement at pivot dup is zero
    # (dup odd: the second pivot of a 2 x 2 step; even: the first; 32: the
    # first pivot of block 2, reached after two pipelined blocks)
    rng = np.random.default_rng(dup)
    J = rng.standard_normal((120, 40))
    J[:, dup] = J[:, src]
    dU, st = _run_ggn(J, rng.standard_normal(120), 0.0, "f64")
    assert st == _lib.ENOTPD
    np.testing.assert_array_equal(dU, np.zeros(40))


@pytest.mark.parametrize("dup", [5, 20, 37])
def test_jacobian_detects_a_late_zero_pivot_of_g(dup):
    # W row dup repeats row 2: G = W W^T is singular from pivot dup on
    rng = np.random.default_rng(dup)
    n, K = 40, 256
    W = rng.standard_normal((n, K))
    W[dup] = W[2]
    R = rng.standard_normal((90, K + 1))
    _, st = _run_jacobian(R, W, "f64")
    assert st == _lib.ERANK


# ---------------------------------------------------------------------------
# a4 + a5 without forming J: gnmppi_ggn_direction
# ---------------------------------------------------------------------------

def _run_direction(R, W, dtype, method, sigma2=0.0, lam=0.0, split=False):
    m, K = R.shape[0], W.shape[1]
    n = W.shape[0]
    Rd, Wd, r0d = padded(R[:, 1:], dtype), padded(W, dtype), to_dev(R[:, 0], dtype)
    code = _lib.F32 if dtype == "f32" else _lib.F64
    work = torch.empty(_lib.gnmppi_ggn_direction_workspace(code, m, n, K), dtype=torch.uint8,
                       device=device())
    dU = to_dev(np.full(n, 7.0), dtype)
    st = torch.full((2,), 99, dtype=torch.int32, device=device())
    if method & 0xff == _lib.JAC_LS:
        # G on a side stream, joined before the half that needs it
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _lib.gnmppi_perturbation_gram(Wd, work, m, st[1:2], K)
        method |= _lib.JAC_GRAM_READY
    else:
        st[1] = 0
        side = None
    if split:
        _lib.gnmppi_ggn_direction(Rd, r0d, Wd, dU, work, method | _lib.JAC_S_ONLY, sigma2, lam,
                                  st[0:1], K=K)
        torch.cuda.current_stream().wait_stream(side)
        _sync()
        assert host(st)[0] == 99  # S_ONLY writes no status
        _lib.gnmppi_ggn_direction(Rd, r0d, Wd, dU, work, method | _lib.JAC_APPLY_ONLY, sigma2, lam,
                                  st[0:1], K=K)
    else:
        if side is not None:
            torch.cuda.current_stream().wait_stream(side)
        _lib.gnmppi_ggn_direction(Rd, r0d, Wd, dU, work, method, sigma2, lam, st[0:1], K=K)
    _sync()
    return host(dU), host(st).tolist()


@pytest.mark.parametrize("case", ["c1", "c2", "chain_f64_ragged", "chain_f32_ragged"])
@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_ggn_direction_ls_matches_the_oracle_step_on_the_ls_jacobian(case, lam):
    # dU = G y with (S^T S + lam G^2) y = -S^T r0 equals the oracle's GGN step
    # on its own LS Jacobian, -(J^T J + lam I)^{-1} J^T r0
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    method = _lib.JAC_LS | (_lib.JAC_BF16X3 if case == "c2" else 0)
    dU, st = _run_direction(R, W, dtype, method, lam=lam)
    assert st == [0, 0]
    assert_parity(dU, ggn.direction(jacobian.ls(R, W), R[:, 0], lam), dtype, "dU (LS, J not formed)")


@pytest.mark.parametrize("case", ["c1", "chain_f32_ragged"])
@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_ggn_direction_mc_matches_the_oracle_step_on_the_mc_jacobian(case, lam):
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    dU, st = _run_direction(R, W, dtype, _lib.JAC_MC, sigma2=sigma * sigma, lam=lam)
    assert st[0] == 0
    ref = ggn.direction(jacobian.mc(R, W, sigma * sigma), R[:, 0], lam)
    assert_parity(dU, ref, dtype, "dU (MC)")


@pytest.mark.parametrize("case", ["c2", "chain_f32_ragged", "chain_f64_ragged"])
def test_ggn_direction_in_two_phases_matches_one_call(case):
    prob, dtype, K, sigma, R, W = _jacobian_inputs(case)
    method = _lib.JAC_LS | (_lib.JAC_BF16X3 if case == "c2" else 0)
    one, st1 = _run_direction(R, W, dtype, method)
    two, st2 = _run_direction(R, W, dtype, method, split=True)
    assert st1 == st2 == [0, 0]
    np.testing.assert_array_equal(two, one)


def test_ggn_direction_at_the_largest_supported_n():
    rng = np.random.default_rng(8)
    n, m, K = 192, 300, 1024
    W = rnd(0.4 * rng.standard_normal((n, K)), "f32")
    A = rng.standard_normal((m, n))
    r0 = rng.standard_normal(m)
    R = rnd(np.concatenate([r0[:, None], r0[:, None] + A @ W], axis=1), "f32")
    dU, st = _run_direction(R, W, "f32", _lib.JAC_LS)
    assert st == [0, 0]
    assert_parity(dU, ggn.direction(jacobian.ls(R, W), R[:, 0]), "f32", "dU (n=192)")


def test_ggn_direction_reports_rank_deficient_perturbations():
    # W row 5 repeats row 2: G and S^T S have exactly equal rows and columns
    # 2 and 5, so both are singular -- the gram's status word says ERANK and
    # the direction's ENOTPD, with dU = 0
    rng = np.random.default_rng(5)
    n, K = 12, 40
    W = rng.standard_normal((n, K))
    W[5] = W[2]
    R = rng.standard_normal((30, K + 1))
    dU, st = _run_direction(R, W, "f64", _lib.JAC_LS)
    assert st == [_lib.ENOTPD, _lib.ERANK]
    np.testing.assert_array_equal(dU, np.zeros(n))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_solver_direction_matches_the_formed_jacobian_path(name):
    # Alg. 1 with J formed (reconstruct + GGN step) and without (one
    # direction call): the same iterates to the dtype's tolerance
    w = wl.get(name)
    dp = DeviceProblem(w.problem, w.dtype)
    out = []
    for form in (True, False):
        g = GNMPPI(dp, w.x0, w.settings, seed=4, max_iters=3, overlap="ahead",
                   form_jacobian=form)
        g.solve(3)
        _sync()
        out.append((host(g.U), g.history(3)))
    assert (out[0][1][2] == 0).all() and (out[1][1][2] == 0).all()
    assert_parity(out[1][0], out[0][0], w.dtype, "U after 3 iterations")
    assert_parity(out[1][1][0], out[0][1][0], w.dtype, "costs")


# ---------------------------------------------------------------------------
# a6: line search + apply
# ---------------------------------------------------------------------------

# 16-lane candidate groups (chains of 9..16 masses) in FP32 and FP64, with
# up to 33 and 40 candidates in one block
@pytest.mark.parametrize("case,L", [("c2", 16), ("c2", 33), ("c1", 16), ("c1", 1), ("c1", 64),
                                    ("chain5_f64", 7), ("chain12_f64", 16), ("chain12_f64", 40)])
def test_line_search_matches_oracle(case, L):
    if case == "c2":
        w = wl.c2()
        prob, x0, dtype = w.problem, w.x0, "f32"
    elif case == "c1":
        w = wl.c1()
        prob, x0, dtype = w.problem, w.x0, "f64"
    elif case == "chain12_f64":
        prob, x0 = wl.chain_problem(n_masses=12, N=9, seed=4)
        dtype = "f64"
    else:
        prob, x0 = wl.chain_problem(n_masses=5, N=11, seed=9)
        dtype = "f64"
    rp = round_problem(prob, dtype)
    rng = np.random.default_rng(L)
    U = rnd(0.1 * rng.standard_normal(prob.n), dtype)
    d = rnd(0.5 * rng.standard_normal(prob.n), dtype)
    alphas = rnd(0.5 ** np.arange(L), dtype)
    x0r = rnd(x0, dtype)
    dp = DeviceProblem(prob, dtype)
    Ud = to_dev(U, dtype)
    Cd = to_dev(np.zeros(L), dtype)
    info = torch.zeros(3, dtype=torch.float64, device=device())
    _lib.gnmppi_line_search(dp, to_dev(x0r, dtype), Ud, to_dev(d, dtype), to_dev(alphas, dtype), Cd, info)
    _sync()
    costs_ref = ocp.cost_from_residual(ocp.residual(rp, x0r, U[:, None] + d[:, None] * alphas[None, :]))
    costs = host(Cd)
    assert_parity(costs, costs_ref, dtype, "candidate costs")
    j = int(np.argmin(costs))  # the device's own decision, checked for validity
    assert costs_ref[j] <= costs_ref.min() * (1 + 10 * TOL[dtype])
    inf = host(info)
    assert int(inf[2]) == j and inf[0] == alphas[j] and inf[1] == costs[j]
    assert_parity(host(Ud), U + alphas[j] * d, dtype, "U_new")


@pytest.mark.parametrize("n_masses", [4, 12])
def test_line_search_skips_nonfinite_candidates(n_masses):
    prob, x0 = wl.chain_problem(n_masses=n_masses, N=6, seed=1)
    dp = DeviceProblem(prob, "f32")
    d = np.full(prob.n, 1e30)  # large steps overflow float32
    alphas = 2.0 ** -np.arange(0, 160, 10, dtype=np.float64)
    Ud = to_dev(np.zeros(prob.n), "f32")
    Cd = to_dev(np.zeros(len(alphas)), "f32")
    info = torch.zeros(3, dtype=torch.float64, device=device())
    st = torch.full((1,), 99, dtype=torch.int32, device=device())
    _lib.gnmppi_line_search(dp, to_dev(x0, "f32"), Ud, to_dev(d, "f32"), to_dev(alphas, "f32"), Cd, info,
                            st)
    _sync()
    costs = host(Cd)
    assert not np.isfinite(costs[0])
    j = int(host(info)[2])
    assert np.isfinite(costs[j]) and costs[j] == np.nanmin(np.where(np.isfinite(costs), costs, np.nan))
    assert int(st.item()) == _lib.OK


@pytest.mark.parametrize("n_masses", [4, 12])
def test_line_search_with_no_finite_candidate_reports_it(n_masses):
    # every candidate overflows: U stays as it was, info = {0, NaN, -1} and the
    # status word says ENONFINITE
    prob, x0 = wl.chain_problem(n_masses=n_masses, N=6, seed=1)
    dp = DeviceProblem(prob, "f32")
    d = np.full(prob.n, 1e30)
    alphas = np.array([1.0, 0.5, 0.25])
    U0 = rnd(0.1 * np.random.default_rng(2).standard_normal(prob.n), "f32")
    Ud = to_dev(U0, "f32")
    Cd = to_dev(np.zeros(len(alphas)), "f32")
    info = torch.zeros(3, dtype=torch.float64, device=device())
    st = torch.zeros(1, dtype=torch.int32, device=device())
    _lib.gnmppi_line_search(dp, to_dev(x0, "f32"), Ud, to_dev(d, "f32"), to_dev(alphas, "f32"), Cd, info,
                            st)
    _sync()
    assert not np.isfinite(host(Cd)).any()
    inf = host(info)
    assert inf[0] == 0.0 and np.isnan(inf[1]) and inf[2] == -1.0
    np.testing.assert_array_equal(host(Ud), U0)
    assert int(st.item()) == _lib.ENONFINITE


@pytest.mark.parametrize("case", ["c2", "c1", "chain5_f64", "chain12_f32_L33"])
def test_line_search_nominal_returns_the_next_nominal_rollout(case):
    # r0, c0 of gnmppi_line_search_nominal are the nominal rollout of the
    # updated controls: r0 bitwise equal to the rollout's column K (the same
    # kernels' arithmetic on the same controls), c0 = 1/2 ||r0||^2 up to the
    # order of the sum; U, C and info as from gnmppi_line_search
    L = 16
    if case == "c2":
        w = wl.c2()
        prob, x0, dtype = w.problem, w.x0, "f32"
    elif case == "c1":
        w = wl.c1()
        prob, x0, dtype = w.problem, w.x0, "f64"
    elif case == "chain5_f64":
        prob, x0 = wl.chain_problem(n_masses=5, N=11, seed=9)
        dtype = "f64"
    else:
        prob, x0 = wl.chain_problem(n_masses=12, N=9, seed=4)
        dtype, L = "f32", 33  # groups of 16 lanes past the last candidate
    rng = np.random.default_rng(7)
    U = rnd(0.1 * rng.standard_normal(prob.n), dtype)
    d = rnd(0.5 * rng.standard_normal(prob.n), dtype)
    alphas = to_dev(rnd(0.5 ** np.arange(L), dtype), dtype)
    dp = DeviceProblem(prob, dtype)
    x0d, dd = to_dev(rnd(x0, dtype), dtype), to_dev(d, dtype)
    m = prob.m
    outs = []
    for nominal in (False, True):
        Ud = to_dev(U, dtype)
        Cd = to_dev(np.zeros(L), dtype)
        info = torch.zeros(3, dtype=torch.float64, device=device())
        st = torch.full((1,), 99, dtype=torch.int32, device=device())
        if nominal:
            Rc = to_dev(np.full(L * m, np.nan), dtype)
            r0 = to_dev(np.full(m, np.nan), dtype)
            c0 = to_dev(np.full(1, np.nan), dtype)
            _lib.gnmppi_line_search_nominal(dp, x0d, Ud, dd, alphas, Rc, r0, c0, Cd, info, st)
        else:
            _lib.gnmppi_line_search(dp, x0d, Ud, dd, alphas, Cd, info, st)
        _sync()
        outs.append((host(Ud), host(Cd), host(info), int(st.item())))
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    # the nominal rollout of the updated controls
    r0_ref = to_dev(np.zeros(m), dtype)
    c0_ref = to_dev(np.zeros(1), dtype)
    _lib.gnmppi_rollout(dp, x0d, Ud, None, 0, None, None, r0_ref, c0_ref)
    _sync()
    np.testing.assert_array_equal(host(r0), host(r0_ref))
    assert_parity(host(c0), host(c0_ref), dtype, "c0")


def test_line_search_nominal_keeps_r0_when_no_candidate_is_finite():
    prob, x0 = wl.chain_problem(n_masses=4, N=6, seed=1)
    dp = DeviceProblem(prob, "f32")
    alphas = to_dev(np.array([1.0, 0.5, 0.25]), "f32")
    U0 = rnd(0.1 * np.random.default_rng(2).standard_normal(prob.n), "f32")
    Ud = to_dev(U0, "f32")
    Rc = to_dev(np.zeros(3 * prob.m), "f32")
    r0 = to_dev(np.full(prob.m, 7.0), "f32")
    c0 = to_dev(np.full(1, 7.0), "f32")
    st = torch.zeros(1, dtype=torch.int32, device=device())
    _lib.gnmppi_line_search_nominal(dp, to_dev(x0, "f32"), Ud, to_dev(np.full(prob.n, 1e30), "f32"),
                                    alphas, Rc, r0, c0, None, None, st)
    _sync()
    assert int(st.item()) == _lib.ENONFINITE
    np.testing.assert_array_equal(host(Ud), U0)
    assert (host(r0) == 7.0).all() and host(c0)[0] == 7.0


@pytest.mark.parametrize("M", [3, 4, 5, 8])
def test_rollout_diverging_sample_leaves_its_neighbours_intact(M):
    # With fewer than 16 lanes per sample, two or four samples share a 16-lane
    # row and the last lane of each reads the next sample's first lane.  Odd
    # columns get controls that overflow float32; every even column (the left
    # neighbour of a diverging one) must still match the oracle.
    prob, x0 = wl.chain_problem(n_masses=M, N=6, seed=M)
    K = 64
    W = rnd(wl.gaussian_perturbations(prob.n, K, 0.2, 3, antithetic=False), "f32")
    W[:, 1::2] = 1e30
    rp, x0r = round_problem(prob, "f32"), rnd(x0, "f32")
    dp = DeviceProblem(prob, "f32")
    Rd = padded(np.zeros((prob.m, K)), "f32")
    Cd = to_dev(np.zeros(K), "f32")
    r0, c0 = to_dev(np.zeros(prob.m), "f32"), to_dev(np.zeros(1), "f32")
    _lib.gnmppi_rollout(dp, to_dev(x0r, "f32"), to_dev(np.zeros(prob.n), "f32"), padded(W, "f32"), K,
                        Rd, Cd, r0, c0)
    _sync()
    R_ref, C_ref = ocp.rollout_batch(rp, x0r, np.zeros(prob.n), W[:, 0::2])
    assert not np.isfinite(host(Cd)[1::2]).any()
    assert_parity(host(Cd)[0::2], C_ref, "f32", "costs of the even columns")
    assert_parity(host(Rd)[:, 0::2], R_ref, "f32", "residuals of the even columns")


# ---------------------------------------------------------------------------
# whole iterations (Alg. 1 and Method C)
# ---------------------------------------------------------------------------

def test_c1_gn_mppi_hits_the_riccati_optimum_in_one_iteration():
    w = wl.c1()
    p = w.problem
    A, B = dynamics.double_integrator_matrices(2, p.dt)
    Q, Rw = np.diag(p.q), np.diag(p.r)
    Ustar, cstar = lqr.riccati_solution(A, B, Q, Rw, Q, p.N, w.x0)
    solver = GNMPPI(DeviceProblem(p, "f64"), w.x0, w.settings, seed=1, max_iters=3)
    solver.solve(3)
    _sync()
    costs, alphas, status = solver.history(3)
    assert (status == 0).all()
    assert abs(costs[0] - cstar) / cstar < 1e-10
    assert abs(costs[2] - cstar) / cstar < 1e-10
    np.testing.assert_allclose(host(solver.U), Ustar, atol=1e-9)
    # the oracle fed the same Philox stream agrees iteration by iteration
    noise = lambda it, s: philox.perturbations(p.n, 256, s, 1, it, "f64")  # noqa: E731
    _, h = solvers.gn_mppi(p, w.x0, np.zeros(p.n), 3, noise, w.settings.sigma0, beta=w.settings.beta,
                           sigma_min=w.settings.sigma_min)
    np.testing.assert_allclose(costs, h.cost, rtol=1e-10)


def test_c2_first_iteration_matches_oracle():
    w = wl.c2()
    p, st = w.problem, w.settings
    rp = round_problem(p, "f32")
    solver = GNMPPI(DeviceProblem(p, "f32"), w.x0, st, seed=1, max_iters=1)
    solver.solve(1)
    _sync()
    costs, alphas, status = solver.history(1)
    assert (status == 0).all()
    noise = lambda it, s: rnd(philox.perturbations(p.n, st.K, s, 1, it, "f32"), "f32")  # noqa: E731
    Uo, h = solvers.gn_mppi(rp, rnd(w.x0, "f32"), np.zeros(p.n), 1, noise, st.sigma0, beta=st.beta,
                            sigma_min=st.sigma_min)
    assert alphas[0] == h.alpha[0]
    assert_parity([costs[0]], [h.cost[0]], "f32", "cost after one iteration")
    assert_parity(host(solver.U), Uo, "f32", "U after one iteration")
    assert costs[0] < ocp.cost(rp, rnd(w.x0, "f32"), np.zeros(p.n))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_nominal_from_the_line_search_keeps_the_trajectory(name):
    # direct-line rolls out without the nominal column after the first step
    # and takes r0 from the line search before it: the same iterates, bit
    # for bit, as direct (r0 is bitwise the rollout's column K)
    w = wl.get(name)
    dp = DeviceProblem(w.problem, w.dtype)
    out = []
    for schedule in ("direct", "direct-line"):
        solver = _solver(dp, w, schedule, seed=9, max_iters=4)
        solver.solve(4)
        _sync()
        out.append((host(solver.U), host(solver.info), host(solver.r0)))
        assert (solver.history(4)[2] == 0).all()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("schedule", list(SCHEDULES))
def test_c1_solver_with_and_without_stream_overlap(schedule):
    w = wl.c1()
    solver = _solver(DeviceProblem(w.problem, "f64"), w, schedule, seed=3, max_iters=2)
    solver.solve(2)
    _sync()
    costs, _, status = solver.history(2)
    assert (status == 0).all()
    with open(os.path.join(os.path.dirname(__file__), "golden", "reference_optima.json")) as f:
        cstar = json.load(f)["c1"]["cstar"]
    assert abs(costs[0] - cstar) / cstar < 1e-10


@pytest.mark.parametrize("schedule", list(SCHEDULES))
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_graph_replays_match_eager_iterations(name, schedule):
    # with overlap the W-only half runs on a side stream ("ahead": one
    # iteration ahead, with its own draw of W and two alternating workspaces;
    # "prefetch": the same, and the main stream uses that W; "same": forked
    # after this iteration's sampler): the same arithmetic as one stream, so
    # bit-identical to eager steps of the same path
    w = wl.get(name)
    dp = DeviceProblem(w.problem, w.dtype)
    eager = _solver(dp, w, "formed" if SCHEDULES[schedule][0] else "direct", seed=5, max_iters=3)
    for it in range(3):
        eager.step(it)
    _sync()
    U_ref, info_ref = host(eager.U), host(eager.info)
    g = _solver(dp, w, schedule, seed=5, max_iters=3)
    graph = g.capture(3)
    for rep in range(3):
        g.U.zero_()                      # fill kernel, outside the graph
        g.info.zero_()
        _lib.gnmppi_rollout(dp, g.x0, g.U, None, 0, None, None, None, g.c0)  # eager work between
        _sync()
        graph.replay()
        _sync()
        np.testing.assert_array_equal(host(g.U), U_ref, err_msg=f"replay {rep}")
        np.testing.assert_array_equal(host(g.info), info_ref, err_msg=f"replay {rep}")
        assert (g.history(3)[2] == 0).all()


def test_plain_mppi_decreases_the_cost_on_c1():
    w = wl.c1()
    solver = PlainMPPI(DeviceProblem(w.problem, "f64"), w.x0, w.settings, max_iters=30)
    for it in range(30):
        solver.step(it)
    solver.final_cost(30)
    _sync()
    cost = host(solver.cost)
    assert (host(solver.status)[:30] == 0).all()
    assert cost[30] < 0.5 * cost[0]
