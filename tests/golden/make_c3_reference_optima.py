"""Writes c3_reference_optima.json: the optimal cost C* of a seeded sample of
the batched workload's instances (1024 chain MPC instances drawn by
``workloads.batch_instances(1024, seed=0)``), computed by the oracle only --
Method A (Sec. 5: GGN with a central finite-difference Jacobian, FP64), 40
iterations from U = 0, as for the single chain workloads in
reference_optima.json.  The batched form's time to a 1e-3 relative cost gap
is judged on these instances against these values.

The sample: 32 distinct instance indices from numpy's default_rng(3); the
first 16 are also the instances solved one at a time for comparison.

Run from the repository root:  python tests/golden/make_c3_reference_optima.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import solvers  # noqa: E402

COUNT, SEED, SAMPLE, SAMPLE_SEED = 1024, 0, 32, 3


def sample_indices():
    return np.random.default_rng(SAMPLE_SEED).choice(COUNT, size=SAMPLE, replace=False)


def compute():
    inst = wl.batch_instances(COUNT, seed=SEED)
    rows = []
    for b in sample_indices():
        p, x0, K = inst[int(b)]
        _, h = solvers.method_a(p, x0, np.zeros(p.n), iters=40)
        rows.append({"index": int(b), "n_masses": p.n_masses, "N": p.N, "K": int(K),
                     "cstar": min(h.cost), "iterations": len(h.cost),
                     "final_grad_norm": h.grad_norm[-1]})
        print(rows[-1], flush=True)
    return {"workload": f"workloads.batch_instances({COUNT}, seed={SEED})",
            "sample": f"{SAMPLE} indices from numpy default_rng({SAMPLE_SEED}).choice({COUNT}, "
                      f"{SAMPLE}, replace=False)",
            "method": "Method A: GGN + central FD, eps=1.49e-8 (oracle.solvers.method_a), 40 iterations",
            "instances": rows}


if __name__ == "__main__":
    res = compute()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_reference_optima.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
