"""Batched GN-MPPI over many independent chain MPC instances of uneven size.

``BatchGNMPPI`` owns the per-instance inputs and outputs (x0, weights,
targets, U, status words, line-search info) and the library workspace; one
``step(it)`` enqueues a whole GN-MPPI iteration for every instance through
``gnmppi_batch_iteration`` (persistent launches per step and shape class),
``capture(iters)`` records iterations into one HIP graph.

``autotune`` is the launch-shape tuner: it times the candidate tunings on the
batch itself and keeps the fastest; results are cached per batch shape in a
JSON file.  The candidates cover the two rollout mappings (a lane group per
sample storing the residuals, then the BF16x3 contraction; or one lane per
sample fused with the contraction on the MFMA) and, per mapping, the grid
sizes of the persistent launches and the k-slices of the separate
contraction.  Every candidate computes the same iteration up to the
summation order of the contraction.
"""
from __future__ import annotations

import ctypes
import hashlib
import itertools
import json
import os
import time

import numpy as np
import torch

from . import _lib

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gnmppi", "batch_autotune.json")

# Candidate tunings: a list of spaces, each the product of its value lists
# (0 = the library's default).  rollout_mode 2 is the fused kernel (the
# contraction fields do not apply to it), 1 the lane-group rollout followed
# by the separate contraction.
TUNING_SPACE = [
    {"rollout_mode": (2,), "small_blocks_per_cu": (8, 16, 32)},
    {"rollout_mode": (1,), "rollout_blocks_per_cu": (16, 32, 64),
     "contract_blocks_per_cu": (16, 32, 64), "contract_ksplit": (1, 2),
     "small_blocks_per_cu": (8, 16, 32)},
]


def _candidates(space):
    """The tunings of a space (dict: product of its value lists) or of a list
    of spaces (their union, in order)."""
    spaces = [space] if isinstance(space, dict) else list(space)
    out = []
    for sp in spaces:
        names = list(sp)
        for values in itertools.product(*(sp[k] for k in names)):
            out.append(dict(zip(names, values)))
    return out


def sigma_schedule(sigma0: float, beta: float, sigma_min: float, it: int) -> float:
    return max(sigma0 * beta ** (0.5 * it), sigma_min)


class BatchGNMPPI:
    """``instances``: list of (Problem, x0, K) with chain problems that share
    dt, k_lin, k_cub and mass.  Settings (sigma schedule, line search) are
    shared by all instances; instance b draws with Philox key seed + b."""

    def __init__(self, instances, settings, seed: int = 1, tuning: dict | None = None,
                 device: str = "cuda"):
        if not instances:
            raise ValueError("empty batch")
        self.dev = torch.device(device)
        self.s = settings
        self.count = len(instances)
        self.problems = [p for p, _, _ in instances]
        p0 = self.problems[0]
        for p in self.problems:
            if (p.model, p.dt, p.k_lin, p.k_cub, p.mass) != (p0.model, p0.dt, p0.k_lin, p0.k_cub, p0.mass):
                raise ValueError("the instances must share the chain model parameters")
        self.shared = _lib.GnmppiProblem(model=p0.model, dtype=_lib.F32, nx=p0.nx, nu=p0.nu, N=p0.N,
                                         n_masses=p0.n_masses, dt=p0.dt, k_lin=p0.k_lin,
                                         k_cub=p0.k_cub, mass=p0.mass, q=None, r=None, x_ref=None)
        # inputs and outputs packed per kind, one slice per instance
        nx = np.array([p.nx for p in self.problems])
        n = np.array([p.n for p in self.problems])
        self.nx_off = np.concatenate([[0], np.cumsum(nx)])
        self.n_off = np.concatenate([[0], np.cumsum(n)])
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.x0 = torch.tensor(np.concatenate([x for _, x, _ in instances]), **f32)
        self.q = torch.tensor(np.concatenate([p.q for p in self.problems]), **f32)
        self.r = torch.tensor(np.concatenate([p.r for p in self.problems]), **f32)
        self.x_ref = torch.tensor(np.concatenate([p.x_ref for p in self.problems]), **f32)
        self.U = torch.zeros(int(self.n_off[-1]), **f32)
        # per instance: Jacobian rank, GGN positive definiteness, line search
        self.status = torch.zeros(self.count, 3, dtype=torch.int32, device=self.dev)
        self.info = torch.zeros(self.count, 3, dtype=torch.float64, device=self.dev)
        arr = (_lib.GnmppiBatchInstance * self.count)()
        for b, (p, _, K) in enumerate(instances):
            a = arr[b]
            a.n_masses, a.N, a.K = p.n_masses, p.N, int(K)
            a.x0 = self.x0[self.nx_off[b]:].data_ptr()
            a.q = self.q[self.nx_off[b]:].data_ptr()
            a.r = self.r[2 * b:].data_ptr()
            a.x_ref = self.x_ref[self.nx_off[b]:].data_ptr()
            a.U = self.U[self.n_off[b]:].data_ptr()
            a.status = self.status[b].data_ptr()
            a.info = self.info[b].data_ptr()
        self.inst = arr
        self.K = np.array([K for _, _, K in instances])
        self.settings = _lib.GnmppiBatchSettings(seed=int(seed), gamma=settings.gamma,
                                                 n_alpha=settings.n_alpha, reserved=0,
                                                 lm_lambda=settings.lm_lambda)
        self.work = None
        self.set_tuning(tuning or {})

    # -- set-up -------------------------------------------------------------
    def _tuning_struct(self, tuning: dict):
        t = _lib.GnmppiBatchTuning()
        for k, v in tuning.items():
            setattr(t, k, int(v))
        return t

    def workspace_bytes(self, tuning: dict) -> int:
        nbytes = _lib.gnmppi_batch_workspace(self.shared, self.count, self.inst, self.settings,
                                             self._tuning_struct(tuning))
        if nbytes == 0:
            raise ValueError("the library rejected the batch (see gnmppi_batch_instance limits)")
        return nbytes

    def set_tuning(self, tuning: dict):
        self.tuning = dict(tuning)
        self.tstruct = self._tuning_struct(self.tuning)
        nbytes = self.workspace_bytes(self.tuning)
        if self.work is None or self.work.numel() < nbytes:
            self.work = None
            torch.cuda.empty_cache()
            self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        _lib.gnmppi_batch_prepare(self.shared, self.count, self.inst, self.settings, self.tstruct,
                                  self.work)

    # -- iterations ---------------------------------------------------------
    def sigma(self, it: int) -> float:
        s = self.s
        return sigma_schedule(s.sigma0, s.beta, s.sigma_min, it)

    def step(self, it: int):
        _lib.gnmppi_batch_iteration(self.shared, self.count, self.inst, self.settings, self.tstruct,
                                    self.work, it, self.sigma(it))

    def capture(self, iters: int, it0: int = 0):
        """One HIP graph holding iterations it0 .. it0 + iters - 1."""
        side = torch.cuda.Stream(device=self.dev)
        side.wait_stream(torch.cuda.current_stream())
        U_save = self.U.clone()
        with torch.cuda.stream(side):  # warm-up outside capture
            self.step(it0)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.U.copy_(U_save)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for it in range(it0, it0 + iters):
                self.step(it)
        return graph

    def controls(self, b: int) -> torch.Tensor:
        return self.U[self.n_off[b]:self.n_off[b + 1]]

    def costs(self) -> np.ndarray:
        """C* of every instance's last line search."""
        return self.info[:, 1].cpu().numpy()


def _batch_key(batch: BatchGNMPPI) -> str:
    shapes = [(p.n_masses, p.N, int(K)) for p, K in zip(batch.problems, batch.K)]
    return hashlib.sha256(json.dumps(shapes).encode()).hexdigest()[:16]


def autotune(batch: BatchGNMPPI, space: dict | None = None, reps: int = 3, cache: str | None = CACHE,
             log=None) -> dict:
    """Times every tuning in ``space`` (the product of its value lists) on one
    iteration of ``batch`` and sets the fastest.  U is restored after each
    trial, so tuning leaves the iterate as it was."""
    space = space or TUNING_SPACE
    key = _batch_key(batch)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if key in known:
            batch.set_tuning(known[key]["tuning"])
            return known[key]
    U0 = batch.U.clone()
    results = []
    for tuning in _candidates(space):
        batch.set_tuning(tuning)
        # timed as graph replays: an eager call also rebuilds the work tables
        # on the host, which a captured iteration never does
        graph = batch.capture(1)
        graph.replay()  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = 0.0
        for _ in range(reps):
            batch.U.copy_(U0)
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1) / reps
        del graph
        results.append((ms, tuning))
        if log:
            log(f"tuning {tuning}: {ms:.3f} ms/iteration")
    batch.U.copy_(U0)
    ms, best = min(results, key=lambda r: r[0])
    batch.set_tuning(best)
    entry = {"tuning": best, "ms_per_iteration": ms, "candidates": len(results),
             "worst_ms": max(r[0] for r in results), "time": time.time()}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[key] = entry
        with open(cache, "w") as f:
            json.dump(known, f)
    return entry
