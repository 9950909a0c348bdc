"""Writes reference_optima.json: the optimal cost C* of each named workload,
computed by the oracle only (Riccati recursion for the linear double
integrator; Method A -- GGN with central finite differences -- for the
nonlinear chain).  Used as the denominator of the relative cost gap.

Run from the repository root:  python tests/golden/make_reference_optima.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import dynamics, lqr, solvers  # noqa: E402


def compute():
    out = {}
    w = wl.c1()
    p = w.problem
    A, B = dynamics.double_integrator_matrices(2, p.dt)
    Q, R = np.diag(p.q), np.diag(p.r)
    _, cstar = lqr.riccati_solution(A, B, Q, R, Q, p.N, w.x0)
    out["c1"] = {"cstar": cstar, "method": "Riccati recursion (oracle.lqr)"}
    for name in ("c2", "c4"):
        w = wl.get(name)
        p = w.problem
        _, h = solvers.method_a(p, w.x0, np.zeros(p.n), iters=40)
        out[name] = {"cstar": min(h.cost), "method": "Method A: GGN + central FD, eps=1.49e-8 (oracle.solvers.method_a)",
                     "iterations": len(h.cost), "final_grad_norm": h.grad_norm[-1]}
    return out


if __name__ == "__main__":
    res = compute()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "reference_optima.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=2)
    print(json.dumps(res, indent=2))
