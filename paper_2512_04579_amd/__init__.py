"""Gauss-Newton accelerated MPPI (arXiv 2512.04579) on AMD Instinct MI355X.

The hot path -- perturbation sampling, single-shooting rollouts with
residuals, the MPPI weighted update, sample-based Jacobian reconstruction,
the GGN step and the parallel line search -- runs in the hand-written HIP
kernels of ``libgnmppi.so`` (C ABI in ``include/gnmppi.h``).  This package
is the thin Python side: the ctypes binding (``_lib``), device-resident
problem data (``problem``) and the outer loops composed of ABI calls
(``solver``).  PyTorch supplies device memory and streams only.
"""
from . import _lib  # noqa: F401
from ._lib import (GnmppiError, gnmppi_abi_version, gnmppi_ggn_step, gnmppi_line_search,  # noqa: F401
                   gnmppi_mppi_update, gnmppi_reconstruct_jacobian, gnmppi_rollout,
                   gnmppi_sample, gnmppi_sigma_points)

__all__ = [
    "GnmppiError", "gnmppi_abi_version", "gnmppi_ggn_step", "gnmppi_line_search",
    "gnmppi_mppi_update", "gnmppi_reconstruct_jacobian", "gnmppi_rollout", "gnmppi_sample",
    "gnmppi_sigma_points",
]
