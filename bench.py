#!/usr/bin/env python3
"""Benchmark of the GN-MPPI hot path on one MI355X.

A step is one GN-MPPI iteration of Alg. 1 over one batch of synthetic input:
sample K perturbations, roll out K + 1 control sequences with residuals,
reconstruct the Jacobian, take the GGN step and run the L-candidate line
search.  Default workload: the 16-mass cubic-spring chain (nx=64, nu=2, RK4
dt=0.05, N=50, K=4096, sigma=0.3, float32).  Inputs are resident in HBM
before the timed region starts.

Printed as one JSON line:
  value            GN-MPPI iterations per second
  sample_steps_per_s  (K + 1 + L) N dynamics evaluations per iteration / time
  time_to_gap_s    wall time to a 1e-3 relative cost gap, GN-MPPI and plain
                   MPPI on the same GPU (C* from the oracle's Method A, stored
                   in tests/golden/reference_optima.json)
  roofline         the dominant kernel's achieved rate against the MI355X peak
  cpu_baseline     the FP64 oracle timed on the host on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GN-MPPI iters/s, sample-steps/s, time-to-1e-3 cost gap vs plain (1 GPU)"
PEAK = {"hbm_GBps": 8000.0, "fp32_TFLOPs": 157.3, "fp64_TFLOPs": 78.6, "bf16_TFLOPs": 2500.0}


def progress(msg: str):
    """One line per finished phase on stderr (the JSON result goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def flops_per_sample_step(prob) -> float:
    """Algorithmic FP operations of one f(x, u) evaluation with its residual
    and cost terms (counted from the model's definition, not the kernel).
    Chain, per RK4 step: 4 right-hand sides of (13 M - 4) flops, 13 nx for the
    stage states and the weighted sum, 2 nx + nu for the residual rows and
    2 (nx + nu) for the cost.  Double integrator: 5 nu for the update."""
    nx, nu = prob.nx, prob.nu
    if prob.model == 2:
        M = prob.n_masses
        return 4 * (13 * M - 4) + 13 * nx + (2 * nx + nu) + 2 * (nx + nu)
    return 5 * nu + (2 * nx + nu) + 2 * (nx + nu)


def algorithmic_work(prob, K: int, L: int, esize: int):
    """Per-launch algorithmic bytes / flops of each library call."""
    m, n, N = prob.m, prob.n, prob.N
    fss = flops_per_sample_step(prob)
    return {
        "rollout": {"bytes": (K + 1) * m * esize + K * n * esize, "flops": (K + 1) * N * fss},
        # the same launch drawing W itself: W written instead of read
        "sample_rollout": {"bytes": (K + 1) * m * esize + K * n * esize,
                           "flops": (K + 1) * N * fss},
        "jacobian": {"bytes": m * K * esize + n * K * esize + m * n * esize,
                     "flops": 2.0 * m * n * K + 2.0 * n * n * K + 2.0 * m * n * n},
        "ggn_step": {"bytes": m * n * esize + m * esize, "flops": 2.0 * m * (n + 1) ** 2 + n ** 3 / 3.0},
        # the direction without J: S and G from one contraction, the normal
        # matrix of [S r0], the solve and dU = G y
        "direction": {"bytes": m * K * esize + n * K * esize + m * esize,
                      "flops": 2.0 * (m + n) * n * K + 2.0 * m * (n + 1) ** 2 + n ** 3 / 3.0
                      + 2.0 * n * n},
        "sample": {"bytes": n * K * esize, "flops": 0.0},
        "line_search": {"bytes": 0, "flops": L * N * fss},
    }


def rollout_traffic(name: str, esize: int):
    """HBM bytes per rollout launch from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when that summary
    was taken for another workload or the kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", f"{name}_rollout_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2512_04579_amd/csrc/rollout.hip", "paper_2512_04579_amd/csrc/common.hpp",
              "paper_2512_04579_amd/csrc/philox.hpp"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if kv.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_model() -> str:
    """The host CPU's model name (lscpu's "Model name", read from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_iterations(w, budget_s: float):
    """GN-MPPI iterations of the oracle on workload w for about budget_s
    seconds; returns (iterations, seconds)."""
    import numpy as np

    import workloads as wl
    from oracle import solvers
    p, st = w.problem, w.settings
    U = np.zeros(p.n)
    its, t0 = 0, time.perf_counter()
    while True:
        noise = lambda it, s: wl.gaussian_perturbations(p.n, st.K, s, 100 + its)  # noqa: E731
        U, _ = solvers.gn_mppi(p, w.x0, U, 1, noise, st.sigma0, beta=st.beta, sigma_min=st.sigma_min,
                               gamma=st.gamma, n_alpha=st.n_alpha)
        its += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            return its, el


def cpu_baseline(w, budget_s: float, single_budget_s: float):
    """The oracle's GN-MPPI iteration timed on the host cores (FP64 NumPy):
    with the BLAS using every host thread, then with one thread."""
    import threadpoolctl

    info = threadpoolctl.threadpool_info()
    blas_threads = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    p, st = w.problem, w.settings
    per_it = (st.K + 1 + st.n_alpha) * p.N
    its, el = _oracle_iterations(w, budget_s)
    out = {"value": its / el, "unit": "iters/s", "cores": int(blas_threads), "kind": "oracle",
           "sample": f"{its} GN-MPPI iterations of the {w.name} workload (K={st.K}, N={p.N}) "
                     f"in FP64 NumPy, {el:.1f} s, BLAS threads = {blas_threads}; host has "
                     f"{os.cpu_count()} logical CPUs",
           "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
           "sample_steps_per_s": its * per_it / el}
    if single_budget_s > 0:
        with threadpoolctl.threadpool_limits(limits=1, user_api="blas"):
            its1, el1 = _oracle_iterations(w, single_budget_s)
        out["single_thread"] = {"value": its1 / el1, "unit": "iters/s", "cores": 1,
                                "sample": f"{its1} iterations, {el1:.1f} s, BLAS limited to one thread",
                                "sample_steps_per_s": its1 * per_it / el1}
    return out


def reference_c3(inst):
    """The oracle's C* of the judged c3 instances (Method A, FP64, written by
    tests/golden/make_c3_reference_optima.py), checked against the shapes of
    the batch being timed."""
    with open(os.path.join(ROOT, "tests", "golden", "c3_reference_optima.json")) as f:
        rows = json.load(f)["instances"]
    for r in rows:
        p, _, K = inst[r["index"]]
        if (p.n_masses, p.N, int(K)) != (r["n_masses"], r["N"], r["K"]):
            raise RuntimeError(f"c3 reference optima do not match instance {r['index']}")
    return rows


def pick_schedule(dp, x0, st, seed: int, iters: int = 50) -> str:
    """The fastest iteration schedule (SCHEDULES in the solver module: the
    direction without J on one stream, with or without the nominal residuals
    handed over by the line search, or J formed with G^{-1} on a side stream
    in one of three orders) for this problem: a graph of ``iters``
    captured iterations per schedule (the length of the timed graphs: "ahead"
    pays for its first iteration's side work once per graph), three replays
    each, the shortest replay counts."""
    import torch

    from paper_2512_04579_amd.solver import make_solver
    best, pick = None, "direct"
    for mode in ("direct", "direct-line", "ahead", "prefetch", "same"):
        solver = make_solver(dp, x0, st, mode, seed=seed, max_iters=iters)
        graph = solver.capture(iters)
        graph.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            if best is None or ms < best:
                best, pick = ms, mode
        del graph, solver
    return pick


def bench_sweep(args):
    """GN-MPPI iterations/s of the chain16 workload at K in {512 .. 8192} and
    N in {20, 50, 80} (graph-timed, 50 iterations per point)."""
    import dataclasses

    import torch

    import workloads as wl
    from paper_2512_04579_amd.problem import DeviceProblem
    from paper_2512_04579_amd.solver import make_solver

    base = wl.c2()
    rows = []
    for N in (20, 50, 80):
        prob, x0 = wl.chain_problem(n_masses=16, N=N, dt=0.05, seed=0)
        dp = DeviceProblem(prob, "f32")
        for K in (512, 1024, 2048, 4096, 8192):
            st = dataclasses.replace(base.settings, K=K)
            mode = pick_schedule(dp, x0, st, seed=1)
            solver = make_solver(dp, x0, st, mode, seed=1, max_iters=51)
            graph = solver.capture(50)
            graph.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 50
            progress(f"sweep N={N} K={K}: {1e3 * ms:.1f} us/iteration")
            rows.append({"N": N, "K": K, "m": prob.m, "n": prob.n, "schedule": mode,
                         "us_per_iter": 1e3 * ms,
                         "iters_per_s": 1e3 / ms,
                         "sample_steps_per_s": (K + 1 + st.n_alpha) * N / (ms * 1e-3)})
            del graph, solver
    return {"metric": METRIC, "unit": "iters/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "chain16 RK4 dt=0.05 scaling sweep over K and N", "name": "c2-sweep"},
            "timed_with": "HIP graph replays of 50 iterations per point", "sweep": rows}


def batched_time_to_gap(args, inst, st, tuning):
    """Time to a 1e-3 gap from U = 0 for the batched form, judged on the
    seeded sample of instances whose C* the oracle computed (Method A, FP64):
    the batch solves all of them, the clock runs until every judged instance
    is within the gap.  Beside it, the same instances one at a time (GN-MPPI
    and plain MPPI)."""
    import numpy as np
    import torch

    from paper_2512_04579_amd.batch import BatchGNMPPI

    ref = reference_c3(inst)
    judged = np.array([r["index"] for r in ref])
    best = np.array([r["cstar"] for r in ref])
    run = BatchGNMPPI(inst, st, seed=1, tuning=tuning)
    graphs = [run.capture(1, it0=it) for it in range(8)]  # one graph per iteration
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True)]
    evs[0].record()
    gaps = []
    for it in range(8):
        graphs[it].replay()
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        evs.append(e)
        gaps.append((run.costs()[judged] - best) / np.abs(best))  # syncs; the times come from the events
    gaps = np.array(gaps)
    del graphs
    t_all = None
    for it in range(len(gaps)):
        if (gaps[it] <= 1e-3).all():
            t_all = evs[0].elapsed_time(evs[it + 1]) * 1e-3
            break
    # the same instances one at a time: GN-MPPI from zero (one captured graph
    # per iteration) and plain MPPI, on the first 16 judged instances;
    # per-instance times summed and scaled to the whole batch
    from paper_2512_04579_amd.problem import DeviceProblem
    from paper_2512_04579_amd.solver import GNMPPI, PlainMPPI
    import dataclasses
    pick = judged[:16]
    t_gn, t_mp, reached_mp = [], [], 0
    for i, b in enumerate(pick):
        p, x0, K = inst[b]
        dp = DeviceProblem(p, "f32")
        stb = dataclasses.replace(st, K=int(K))
        cst = best[i]
        g = GNMPPI(dp, x0, stb, seed=1 + int(b), max_iters=8)
        gr = [g.capture(1, it0=it) for it in range(8)]
        g.U.zero_()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tb = None
        for it in range(8):
            gr[it].replay()
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            c = g.info[it, 1].item()
            if (c - cst) / abs(cst) <= 1e-3:
                tb = e0.elapsed_time(e) * 1e-3
                break
        t_gn.append(tb)
        del gr, g
        mp = PlainMPPI(dp, x0, stb, seed=200 + int(b), max_iters=args.mppi_iters)
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record()
        evs = []
        for it in range(args.mppi_iters):
            mp.step(it)
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            evs.append(e)
        mp.final_cost(args.mppi_iters)
        torch.cuda.synchronize()
        mc = mp.cost.double().cpu().numpy()
        hit = np.nonzero((mc[1:] - cst) / abs(cst) <= 1e-3)[0]
        if hit.size:
            reached_mp += 1
            t_mp.append(e0.elapsed_time(evs[hit[0]]) * 1e-3)
    gn_ok = [t for t in t_gn if t is not None]
    sequential = {
        "sample": f"{len(pick)} of the {len(judged)} judged instances, times summed and scaled by "
                  f"{len(inst)}/{len(pick)}",
        "gn_mppi_single_instance_s": (sum(gn_ok) * len(inst) / len(gn_ok)) if gn_ok else None,
        "gn_mppi_reached": f"{len(gn_ok)}/{len(pick)} within 8 iterations",
        "plain_mppi_single_instance_s": (sum(t_mp) * len(inst) / len(t_mp)) if t_mp else None,
        "plain_mppi_reached": f"{reached_mp}/{len(pick)} within {args.mppi_iters} iterations "
                              f"(c2's plain-MPPI temperature and sigma schedule)",
    }
    return {"all_judged_instances": t_all, "gap_threshold": 1e-3,
            "one_instance_at_a_time": sequential,
            "median_gap_per_iter": [float(np.median(g)) for g in gaps],
            "max_gap_per_iter": [float(np.max(g)) for g in gaps],
            "cstar": f"oracle Method A (FP64) on {len(judged)} seeded instances "
                     "(tests/golden/c3_reference_optima.json)",
            "judged_instances": [int(b) for b in judged]}


def bench_batched(args, steps: int, warmup: int, tune: bool):
    """The batched form: ``--batch-count`` chain instances with M in 4..16,
    N in 20..80 and K in {512, 1024, 2048, 4096} (seeded), one GN-MPPI
    iteration for all of them per step, timed as HIP-graph replays after the
    launch-shape autotuner has picked its tuning."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2512_04579_amd.batch import BatchGNMPPI, autotune

    inst = wl.batch_instances(args.batch_count, seed=0)
    st = wl.c2().settings
    L = st.n_alpha
    batch = BatchGNMPPI(inst, st, seed=1, tuning=json.loads(args.batch_tuning or "{}"))
    tuned = autotune(batch, cache=None, log=progress) if tune else {
        "tuning": args.batch_tuning or "library default (an autotuner pick for this batch)"}
    chunk = max(1, min(steps, 10))
    reps = max(1, steps // chunk)
    steps = reps * chunk
    graph = batch.capture(chunk)
    for _ in range(max(1, warmup // chunk)):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    status = batch.status.cpu().numpy()
    assert (status == 0).all(), f"device status words: {np.unique(status)}"
    Ks = np.array([K for _, _, K in inst])
    Ns = np.array([p.N for p, _, _ in inst])
    ms_ = np.array([p.m for p, _, _ in inst])
    ns = np.array([p.n for p, _, _ in inst])
    sample_steps = float(((Ks + 1 + L) * Ns).sum())
    # algorithmic HBM bytes of one iteration: R written by the rollout and read
    # by the sample contraction, W written by the sampler and read twice
    r_bytes = float((ms_ * Ks * 4).sum())
    w_bytes = float((ns * Ks * 4).sum())
    iter_bytes = 2 * r_bytes + 3 * w_bytes
    gbps = iter_bytes / (ms * 1e-3) / 1e9

    del graph
    ttg = batched_time_to_gap(args, inst, st, batch.tuning) if not args.no_time_to_gap else None
    return {
        "metric": METRIC,
        "value": 1e3 / ms,
        "unit": "batched iters/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(inst)} chain MPC instances, M 4..16, N 20..80, "
                               f"K in {{512,1024,2048,4096}}, batched GN-MPPI iteration", "name": "c3",
                   "instances": len(inst), "sum_m": int(ms_.sum()), "sum_n": int(ns.sum()),
                   "sum_K": int(Ks.sum()), "tuning": batch.tuning},
        "instance_iters_per_s": len(inst) * 1e3 / ms,
        "sample_steps_per_s": sample_steps / (ms * 1e-3),
        "timed_with": f"HIP graph replays of {chunk} batched iterations",
        "roofline": {"kernel": "whole batched iteration", "bound": "hbm", "achieved": gbps,
                     "peak": PEAK["hbm_GBps"], "unit": "GB/s", "frac": gbps / PEAK["hbm_GBps"],
                     "traffic": None, "algorithmic_bytes": iter_bytes},
        "autotune": tuned,
        "time_to_gap_s": ttg,
    }


def bench_single(w, args, steps_req: int, warmup: int):
    """One workload through the single-instance solver: graph-timed
    iterations, per-call times, the rollout kernel's roofline and the time to
    a 1e-3 cost gap against the oracle's C*."""
    import numpy as np
    import torch

    from paper_2512_04579_amd import _lib
    from paper_2512_04579_amd.problem import DeviceProblem
    from paper_2512_04579_amd.solver import GNMPPI, PlainMPPI, make_solver

    p, st = w.problem, w.settings
    dp = DeviceProblem(p, w.dtype)
    esize = 4 if w.dtype == "f32" else 8
    # The timed region replays HIP graphs of `chunk` captured iterations, so the
    # host enqueues one launch per chunk instead of ~12 kernels per iteration.
    chunk = min(steps_req, args.graph_chunk)
    reps = max(1, steps_req // chunk)
    steps = reps * chunk
    # The graphs run the fastest of the iteration schedules (the direction
    # without J on one stream, or J formed with G^{-1} on a side stream);
    # eager launches run the direction without J.
    if args.eager:
        schedule = "direct"
    elif args.schedule == "auto":
        schedule = pick_schedule(dp, w.x0, st, seed=w.noise_seed, iters=chunk)
    else:
        schedule = args.schedule
    progress(f"iteration schedule: {schedule}")
    solver = make_solver(dp, w.x0, st, schedule, seed=w.noise_seed, max_iters=chunk + 1)
    graph = solver.capture(chunk) if not args.eager else None
    for _ in range(max(1, warmup // chunk)):
        graph.replay() if graph else [solver.step(it) for it in range(chunk)]
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_start.record()
    for _ in range(reps):
        if graph:
            graph.replay()
        else:
            for it in range(chunk):
                solver.step(it)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_end)
    ms_per_step = ms_total / steps
    _, _, status = solver.history(chunk)
    assert (status == 0).all(), f"device status words: {np.unique(status)}"

    # Per-call durations: HIP events around each library call of eager
    # iterations.  A device-side spin before each iteration holds the stream
    # until the host has enqueued the whole iteration, so the host's launch
    # gaps stay out of the per-call times.  Then the rollout kernel alone in a
    # back-to-back loop on the launch stream gives the roofline's duration.
    # (a single-stream solver, so that every call's time holds all its work)
    solver = GNMPPI(dp, w.x0, st, seed=w.noise_seed, max_iters=chunk + 1)
    marks = {}
    for it in range(chunk):
        torch.cuda._sleep(1_000_000)
        solver.step(it, marks)
        torch.cuda.synchronize()
    per_call_us = {k: 1e3 * float(np.median([a.elapsed_time(b) for a, b in v])) for k, v in marks.items()}
    # the launch that the iteration runs: W drawn inside the rollout
    Kc = solver.K
    Wv, Rv = solver.W[:, :Kc], solver.R[:, :Kc]

    def rollout_launch():
        _lib.gnmppi_sample_rollout(dp, solver.x0, solver.U, Wv, solver.sigma(0), solver.seed, 0, Kc,
                                   antithetic=st.antithetic, R=Rv, r0=solver.r0, c0=solver.c0)

    for _ in range(3):
        rollout_launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.kernel_reps):
        rollout_launch()
    e1.record()
    torch.cuda.synchronize()
    rollout_us = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
    per_call_us["rollout_kernel"] = rollout_us

    K, L, N = solver.K, st.n_alpha, p.N
    work = algorithmic_work(p, K, L, esize)
    fp_peak = PEAK["fp32_TFLOPs"] if esize == 4 else PEAK["fp64_TFLOPs"]
    calls = {}
    for name, us in per_call_us.items():
        wk = work["rollout" if name == "rollout_kernel" else name]
        t = us * 1e-6
        entry = {"us": us, "GBps": wk["bytes"] / t / 1e9, "TFLOPs": wk["flops"] / t / 1e12}
        entry["hbm_frac"] = entry["GBps"] / PEAK["hbm_GBps"]
        entry["fp_frac"] = entry["TFLOPs"] / fp_peak
        calls[name] = entry
    # Roofline of the rollout kernel: the largest single launch of the
    # iteration and the one library call that is exactly one kernel, so its
    # HIP-event time on the launch stream is the kernel's duration.
    ro = calls["rollout_kernel"]
    roofline = {"kernel": "rollout_chain_split_kernel" if p.model == 2 else "rollout_di_kernel",
                "bound": "hbm", "achieved": ro["GBps"], "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                "frac": ro["hbm_frac"], "traffic": rollout_traffic(w.name, esize),
                "algorithmic_bytes": work["rollout"]["bytes"], "launch_us": ro["us"],
                "alu_TFLOPs": ro["TFLOPs"], "alu_frac": ro["fp_frac"]}

    result = {
        "metric": METRIC,
        "value": steps / (ms_total * 1e-3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": w.description, "name": w.name, "nx": p.nx, "nu": p.nu, "N": N, "K": K,
                   "m": p.m, "n": p.n, "line_search_candidates": L, "jacobian": st.jacobian,
                   "contraction": st.contraction, "schedule": schedule},
        "sample_steps_per_s": steps * (K + 1 + L) * N / (ms_total * 1e-3),
        "host_wall_s": wall,
        "per_call": calls,
        "iteration_over_rollout": ms_per_step * 1e3 / per_call_us["rollout_kernel"],
        "timed_with": "eager launches" if args.eager else
        f"HIP graph replays of {chunk} iterations, schedule {schedule!r}"
        + (" (the fastest of four timed at start-up)" if args.schedule == "auto" else ""),
        "roofline": roofline,
    }

    progress("timed region, per-call timing and roofline done")
    if not args.no_time_to_gap:
        with open(os.path.join(ROOT, "tests", "golden", "reference_optima.json")) as f:
            cstar = json.load(f)[w.name]["cstar"]
        g = GNMPPI(dp, w.x0, st, seed=w.noise_seed + 100, max_iters=st.iters)
        torch.cuda.synchronize()
        evs = g.solve(st.iters, events=True)
        torch.cuda.synchronize()
        costs, _, _ = g.history(st.iters)
        gaps = (costs - cstar) / abs(cstar)
        hit = np.nonzero(gaps <= 1e-3)[0]
        t_gn = evs[0].elapsed_time(evs[hit[0] + 1]) * 1e-3 if hit.size else None
        # Method E: the same solver driven by the 2n-point sigma-point set
        ge = GNMPPI(dp, w.x0, st, sampler="sigma_points", max_iters=st.iters)
        torch.cuda.synchronize()
        eevs = ge.solve(st.iters, events=True)
        torch.cuda.synchronize()
        ecosts, _, _ = ge.history(st.iters)
        egaps = (ecosts - cstar) / abs(cstar)
        ehit = np.nonzero(egaps <= 1e-3)[0]
        t_e = eevs[0].elapsed_time(eevs[ehit[0] + 1]) * 1e-3 if ehit.size else None
        # learned warm start (chain workload with a trained network): the
        # network's proposal or U = 0, whichever rolls out cheaper, then the
        # same solver; the clock starts before the network's forward pass
        warm = None
        from paper_2512_04579_amd import warmstart
        if p.model == 2 and p.N == 50 and os.path.exists(warmstart.DEFAULT_WEIGHTS):
            net = warmstart.WarmStartNet.load(warmstart.DEFAULT_WEIGHTS)
            gw = GNMPPI(dp, w.x0, st, seed=w.noise_seed + 100, max_iters=st.iters)
            warmstart.start_controls(net, dp, gw.x0, gw.U)  # first-call set-up outside the clock
            torch.cuda.synchronize()
            ws0 = torch.cuda.Event(enable_timing=True)
            ws0.record()
            winfo = warmstart.start_controls(net, dp, gw.x0, gw.U)
            ws1 = torch.cuda.Event(enable_timing=True)
            ws1.record()
            wevs = gw.solve(st.iters, events=True)
            torch.cuda.synchronize()
            wcosts, _, _ = gw.history(st.iters)
            which = "network" if winfo[0].item() == 1.0 else "zero"
            g0 = (winfo[1].item() - cstar) / abs(cstar)
            wgaps = (wcosts - cstar) / abs(cstar)
            whit = np.nonzero(wgaps <= 1e-3)[0]
            if g0 <= 1e-3:
                t_w, it_w = ws0.elapsed_time(ws1) * 1e-3, 0
            elif whit.size:
                t_w, it_w = ws0.elapsed_time(wevs[whit[0] + 1]) * 1e-3, int(whit[0] + 1)
            else:
                t_w, it_w = None, None
            warm = {"time_s": t_w, "iters": it_w, "start": which, "start_gap": float(g0),
                    "start_seconds": ws0.elapsed_time(ws1) * 1e-3, "final_gap": float(wgaps[-1]),
                    "gap_after_1_iter": float(wgaps[0]), "zero_start_gap_after_1_iter": float(gaps[0]),
                    "training": getattr(net, "meta", {})}
        mp = PlainMPPI(dp, w.x0, st, seed=w.noise_seed + 200, max_iters=args.mppi_iters)
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record()
        mevs = []
        for it in range(args.mppi_iters):
            mp.step(it)
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            mevs.append(e)
        mp.final_cost(args.mppi_iters)
        torch.cuda.synchronize()
        mcost = mp.cost.double().cpu().numpy()  # mcost[i] = C(U_i), before update i
        mgap = (mcost - cstar) / abs(cstar)
        mhit = np.nonzero(mgap[1:] <= 1e-3)[0]
        t_mp = e0.elapsed_time(mevs[mhit[0]]) * 1e-3 if mhit.size else None
        result["time_to_gap_s"] = {"gn_mppi": t_gn, "gn_mppi_iters": int(hit[0] + 1) if hit.size else None,
                                   "gn_mppi_sigma_points": t_e,
                                   "gn_mppi_sigma_points_iters": int(ehit[0] + 1) if ehit.size else None,
                                   "gn_mppi_sigma_points_final_gap": float(egaps[-1]),
                                   "gn_mppi_warm_start": warm,
                                   "plain_mppi": t_mp,
                                   "plain_mppi_iters": int(mhit[0] + 1) if mhit.size else None,
                                   "gn_mppi_final_gap": float(gaps[-1]),
                                   "plain_mppi_final_gap": float(mgap[-1]),
                                   "plain_mppi_iters_run": args.mppi_iters, "cstar": cstar,
                                   "gap_threshold": 1e-3}

    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"],
                    help="c3 = 1024 uneven chain instances through the batched iteration")
    ap.add_argument("--batch-count", type=int, default=1024, help="instances of the c3 workload")
    ap.add_argument("--sweep", action="store_true",
                    help="chain16 scaling curves: iterations/s at K in 512..8192 and N in 20, 50, 80")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle timing")
    ap.add_argument("--cpu-single-budget", type=float, default=8.0,
                    help="seconds of single-thread oracle timing (0: skip)")
    ap.add_argument("--no-extra", action="store_true",
                    help="c2 only: leave out the c4 and c3 objects of the default line")
    ap.add_argument("--batch-tuning", default="",
                    help='c3: tuning fields as JSON, e.g. {"rollout_mode": 2} (default: the library\'s)')
    ap.add_argument("--autotune", action="store_true",
                    help="--workload c3: run the launch-shape autotuner before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-gap", action="store_true")
    ap.add_argument("--mppi-iters", type=int, default=1500)
    ap.add_argument("--graph-chunk", type=int, default=50, help="iterations per captured graph")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graphs")
    ap.add_argument("--schedule", choices=("auto", "direct", "direct-line", "formed", "ahead",
                                           "prefetch", "same"),
                    default="auto",
                    help="iteration schedule of the graphs: direct = the GGN direction without "
                         "forming J, one stream; direct-line = the same with the nominal residuals "
                         "from the line search; formed = J formed, one stream; ahead / prefetch "
                         "/ same = J formed, G^{-1} on a side stream (auto: the fastest of "
                         "direct, direct-line, ahead, prefetch, same)")
    ap.add_argument("--kernel-reps", type=int, default=50, help="rollout launches for the roofline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "described but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as wl
    from paper_2512_04579_amd import _lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    _lib.load()
    if args.copy_calibration:
        a = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")  # 256 MiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4,
                          "launches": 5}))
        return

    if args.workload == "c3":
        print(json.dumps(bench_batched(args, args.steps, args.warmup, tune=args.autotune)))
        return
    if args.sweep:
        print(json.dumps(bench_sweep(args)))
        return
    w = wl.get(args.workload)
    result = bench_single(w, args, args.steps, args.warmup)
    if args.workload == "c2" and not args.no_extra:
        # the precision split (c4) and the batched form (c3) in the same line:
        # graph-timed iterations and time to the 1e-3 gap of each
        progress("c4: precision split")
        c4 = bench_single(wl.c4(), args, 50, 10)
        for key in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data",
                    "host_wall_s"):
            c4.pop(key, None)
        result["c4"] = c4
        progress("c3: batched form (library default tuning)")
        c3 = bench_batched(args, steps=10, warmup=10, tune=False)
        for key in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            c3.pop(key, None)
        result["c3"] = c3
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, args.cpu_single_budget)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
