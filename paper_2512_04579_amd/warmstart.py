"""Learned warm start for GN-MPPI on the chain instance.

A perceptron 4M -> 256 -> 256 -> N nu (GELU, bfloat16 weights, float32
accumulation) maps the initial state x0 to a control sequence U0(x0), from
which GN-MPPI (Alg. 1, unchanged) starts instead of from zero.  The network
is trained on (x0, U*) pairs that the solver itself produces: GN-MPPI run
from zero on initial states drawn like the instance's own.  Forward pass,
backpropagation and Adam run in the library's kernels (gnmppi_mlp_*);
PyTorch only holds the tensors.

The zero start stays both the fallback and the judge: ``start_controls``
rolls out the proposal and U = 0 in one launch and keeps whichever costs
less, and the gain is measured against GN-MPPI from zero.

Command line (one GPU):
    python -m paper_2512_04579_amd.warmstart --pairs 100000 --epochs 40 \
        --out paper_2512_04579_amd/data/warmstart_chain16.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _lib
from .problem import DeviceProblem
from .solver import GNMPPI

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "warmstart_chain16.npz")


class WarmStartNet:
    """The perceptron with its float32 master weights, bfloat16 compute copy
    and Adam moments; inputs and outputs are standardised with the training
    set's statistics, which ``inference_params`` folds into W1, b1, W3, b3."""

    def __init__(self, n_in: int, n_out: int, n_hidden: int = 256, seed: int = 0,
                 device: str = "cuda"):
        self.dims = (int(n_in), int(n_hidden), int(n_out))
        self.device = torch.device(device)
        I, H, O = self.dims
        rng = np.random.default_rng(seed)
        parts = [rng.standard_normal((H, I)) / np.sqrt(I), np.zeros(H),
                 rng.standard_normal((H, H)) / np.sqrt(H), np.zeros(H),
                 rng.standard_normal((O, H)) / np.sqrt(H), np.zeros(O)]
        flat = np.concatenate([p.reshape(-1) for p in parts])
        assert flat.size == _lib.gnmppi_mlp_param_count(I, H, O)
        self.master = torch.tensor(flat, dtype=torch.float32, device=self.device)
        self.params = self.master.to(torch.bfloat16)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.step = 0
        self.x_mean, self.x_std = np.zeros(I), np.ones(I)
        self.y_mean, self.y_std = np.zeros(O), np.ones(O)
        self._work = {}
        self._folded = None
        self._alpha = {}

    # -- helpers -------------------------------------------------------------
    def _workspace(self, batch: int) -> torch.Tensor:
        if batch not in self._work:
            nbytes = _lib.gnmppi_mlp_workspace(*self.dims, batch)
            self._work[batch] = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._work[batch]

    def _split(self, flat):
        I, H, O = self.dims
        sizes = [H * I, H, H * H, H, O * H, O]
        out, o = [], 0
        for s in sizes:
            out.append(flat[o:o + s])
            o += s
        W1, b1, W2, b2, W3, b3 = out
        return W1.reshape(H, I), b1, W2.reshape(H, H), b2, W3.reshape(O, H), b3

    # -- training ------------------------------------------------------------
    def fit(self, X, Y, epochs: int, batch: int = 1024, lr: float = 1e-3, lr_final: float = 1e-5,
            seed: int = 0, log=None):
        """Adam on L = |net(x) - y|^2 / (2 O) over standardised data; the step
        size decays geometrically from ``lr`` to ``lr_final``.  Returns the
        mean training loss of every epoch."""
        X = np.asarray(X, dtype=np.float64)
        Y = np.asarray(Y, dtype=np.float64)
        self.x_mean, self.x_std = X.mean(0), X.std(0)
        self.y_mean, self.y_std = Y.mean(0), Y.std(0)
        self.x_std[self.x_std < 1e-6] = 1.0  # constant features (the end mass starts at rest)
        self.y_std[self.y_std < 1e-6] = 1.0
        Xd = torch.tensor((X - self.x_mean) / self.x_std, dtype=torch.float32, device=self.device)
        Yd = torch.tensor((Y - self.y_mean) / self.y_std, dtype=torch.float32, device=self.device)
        count = X.shape[0]
        batch = min(batch, count)
        nb = count // batch
        work = self._workspace(batch)
        losses = torch.zeros(epochs, nb, dtype=torch.float32, device=self.device)
        rng = np.random.default_rng(seed)
        total = epochs * nb
        decay = (lr_final / lr) ** (1.0 / max(total - 1, 1))
        xb = torch.empty(batch, self.dims[0], dtype=torch.float32, device=self.device)
        yb = torch.empty(batch, self.dims[2], dtype=torch.float32, device=self.device)
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = torch.tensor(rng.permutation(count), device=self.device)
            for b in range(nb):
                idx = perm[b * batch:(b + 1) * batch]
                torch.index_select(Xd, 0, idx, out=xb)
                torch.index_select(Yd, 0, idx, out=yb)
                _lib.gnmppi_mlp_backward(self.dims, self.params, xb, yb, losses[ep, b:b + 1],
                                         self.grad, work)
                self.step += 1
                _lib.gnmppi_mlp_adam(self.master, self.params, self.grad, self.m, self.v,
                                     lr * decay ** (self.step - 1), self.step)
            if log is not None and (ep + 1) % max(1, epochs // 10) == 0:
                log(f"epoch {ep + 1}/{epochs}: loss {losses[ep].mean().item():.3e} "
                    f"({time.perf_counter() - t0:.1f} s)")
        self._folded = None
        return losses.mean(1).cpu().numpy()

    # -- inference -----------------------------------------------------------
    def inference_params(self) -> torch.Tensor:
        """bfloat16 parameters acting on raw x0 and giving raw U: the input
        standardisation folded into W1, b1 and the output scaling into W3, b3
        (computed in float64 from the master weights)."""
        if self._folded is None:
            W1, b1, W2, b2, W3, b3 = self._split(self.master.double().cpu().numpy())
            W1f = W1 / self.x_std[None, :]
            b1f = b1 - W1f @ self.x_mean
            W3f = self.y_std[:, None] * W3
            b3f = self.y_std * b3 + self.y_mean
            flat = np.concatenate([a.reshape(-1) for a in (W1f, b1f, W2, b2, W3f, b3f)])
            self._folded = torch.tensor(flat, dtype=torch.float32, device=self.device).to(torch.bfloat16)
        return self._folded

    def predict(self, X: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """U0 for each row of X (B x 4M float32 on the device)."""
        B = X.shape[0]
        if out is None:
            out = torch.empty(B, self.dims[2], dtype=torch.float32, device=self.device)
        _lib.gnmppi_mlp_forward(self.dims, self.inference_params(), X, out, self._workspace(B))
        return out

    # -- persistence ---------------------------------------------------------
    def save(self, path: str, meta: dict | None = None):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez(path, dims=np.array(self.dims), master=self.master.cpu().numpy(),
                 x_mean=self.x_mean, x_std=self.x_std, y_mean=self.y_mean, y_std=self.y_std,
                 meta=np.array(json.dumps(meta or {})))

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "WarmStartNet":
        with np.load(path, allow_pickle=False) as f:
            I, H, O = (int(v) for v in f["dims"])
            net = cls(I, O, H, device=device)
            net.master.copy_(torch.from_numpy(f["master"]))
            net.params = net.master.to(torch.bfloat16)
            for k in ("x_mean", "x_std", "y_mean", "y_std"):
                setattr(net, k, f[k].astype(np.float64))
            net.meta = json.loads(str(f["meta"]))
        return net


def start_controls(net: WarmStartNet, dprob: DeviceProblem, x0: torch.Tensor, U: torch.Tensor,
                   info: torch.Tensor | None = None) -> torch.Tensor:
    """Writes the start U of GN-MPPI for initial state x0 into ``U``: the
    network's proposal, or zero if the proposal's rollout costs more (or is
    not finite).  Done on the device without a host round trip: the line
    search of Eq. (15) from U = 0 along the proposal with step lengths
    {1, 0} evaluates both candidates in one launch and applies the cheaper
    (ties go to the proposal).  Returns ``info`` = {alpha*, C*, j*}
    (alpha* = 1: the network's start was taken)."""
    prop = net.predict(x0.reshape(1, -1).to(torch.float32))[0]
    U.zero_()
    key = (U.dtype, U.device)
    if key not in net._alpha:  # kept on the device: no host copy per call
        net._alpha[key] = torch.tensor([1.0, 0.0], dtype=U.dtype, device=U.device)
    if info is None:
        info = torch.empty(3, dtype=torch.float64, device=U.device)
    _lib.gnmppi_line_search(dprob, x0, U, prop.to(U.dtype), net._alpha[key], None, info)
    return info


def solve_pairs(workload, X0: np.ndarray, iters: int, seed: int | None = None, log=None):
    """U* for every initial state in X0: GN-MPPI from zero, ``iters``
    iterations replayed from one captured graph.  Returns (U*, final cost,
    worst status word) as numpy arrays."""
    p, st = workload.problem, workload.settings
    dp = DeviceProblem(p, workload.dtype)
    solver = GNMPPI(dp, workload.x0, st, seed=workload.noise_seed if seed is None else seed,
                    max_iters=iters)
    graph = solver.capture(iters)
    count = X0.shape[0]
    Xd = torch.tensor(X0, dtype=solver.x0.dtype, device=dp.device)
    Us = torch.empty(count, p.n, dtype=solver.U.dtype, device=dp.device)
    costs = torch.empty(count, dtype=torch.float64, device=dp.device)
    worst = torch.zeros(count, dtype=torch.int32, device=dp.device)
    t0 = time.perf_counter()
    for i in range(count):
        solver.x0.copy_(Xd[i])
        solver.U.zero_()
        graph.replay()
        Us[i].copy_(solver.U)
        costs[i].copy_(solver.info[iters - 1, 1])
        worst[i].copy_(torch.amin(solver.status[:iters]))
        if log is not None and (i + 1) % max(1, count // 10) == 0:
            torch.cuda.synchronize()
            log(f"solved {i + 1}/{count} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return Us.double().cpu().numpy(), costs.cpu().numpy(), worst.cpu().numpy()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--pairs", type=int, default=100000)
    ap.add_argument("--iters", type=int, default=4, help="GN-MPPI iterations per training solve")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as wl

    log = lambda s: print(s, flush=True)  # noqa: E731
    w = wl.c2()
    X0 = wl.chain_initial_states(args.pairs, args.seed, w.problem.n_masses)
    t0 = time.perf_counter()
    U, costs, worst = solve_pairs(w, X0, args.iters, log=log)
    t_data = time.perf_counter() - t0
    ok = worst == 0
    log(f"{ok.sum()} of {len(ok)} solves without a device status; {t_data:.1f} s")
    net = WarmStartNet(w.problem.nx, w.problem.n, seed=args.seed)
    t1 = time.perf_counter()
    hist = net.fit(X0[ok], U[ok], args.epochs, args.batch, args.lr, log=log)
    t_train = time.perf_counter() - t1
    meta = {"pairs": int(ok.sum()), "solver_iters": args.iters, "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "final_loss": float(hist[-1]),
            "data_seconds": t_data, "train_seconds": t_train, "seed": args.seed}
    net.save(args.out, meta)
    log(json.dumps(meta))


if __name__ == "__main__":
    main()
