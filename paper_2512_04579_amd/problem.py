"""Device-resident problem description for the C ABI.

Holds the ``gnmppi_problem`` struct together with the torch tensors its
pointers refer to (diagonal weights and tracking target), so they stay alive
as long as the problem is used.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

TORCH_DTYPES = {"f32": torch.float32, "f64": torch.float64}
ABI_DTYPES = {"f32": _lib.F32, "f64": _lib.F64}


class DeviceProblem:
    def __init__(self, problem, dtype: str = "f32", device: str = "cuda"):
        self.host = problem
        self.dtype = dtype
        self.tdtype = TORCH_DTYPES[dtype]
        self.device = torch.device(device)
        as_dev = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64)).to(  # noqa: E731
            device=self.device, dtype=self.tdtype).contiguous()
        self.q = as_dev(problem.q)
        self.r = as_dev(problem.r)
        self.x_ref = as_dev(problem.x_ref)
        self.c = _lib.GnmppiProblem(
            model=problem.model, dtype=ABI_DTYPES[dtype], nx=problem.nx, nu=problem.nu,
            N=problem.N, n_masses=problem.n_masses, dt=problem.dt, k_lin=problem.k_lin,
            k_cub=problem.k_cub, mass=problem.mass, q=self.q.data_ptr(), r=self.r.data_ptr(),
            x_ref=self.x_ref.data_ptr())

    @property
    def n(self) -> int:
        return self.host.n

    @property
    def m(self) -> int:
        return self.host.m

    def tensor(self, a) -> torch.Tensor:
        return torch.as_tensor(np.asarray(a, dtype=np.float64)).to(
            device=self.device, dtype=self.tdtype).contiguous()
