"""The allocation-free GGN step (gnmppi_ggn_step_noalloc: scratch in the
library's fixed device array) against the workspace form gnmppi_ggn_step,
called through the C ABI on the same inputs: two calls in a row, the second
smaller, in both element types.  Both run the same kernels in the same order,
so the directions must agree bit for bit; each is also checked against the
oracle's GGN direction (Eq. (13)) at the element type's bar.
"""
import numpy as np
import pytest
import torch

from _parity import assert_parity, device, host, rnd, to_dev
from oracle import ggn
from paper_2512_04579_amd import _lib

pytestmark = pytest.mark.gpu

CODE = {"f32": _lib.F32, "f64": _lib.F64}


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_ggn_step_matches_the_workspace_call(dtype):
    dev = device()
    tdt = torch.float32 if dtype == "f32" else torch.float64
    # the c2 shape, then a smaller ragged one (the scratch keeps the first
    # call's contents; nothing of it may leak into the second)
    for m, n, lam, seed in [(3300, 100, 0.0, 1), (700, 37, 0.1, 2)]:
        rng = np.random.default_rng(seed)
        J = rnd(rng.standard_normal((m, n)), dtype)
        r0 = rnd(rng.standard_normal(m), dtype)
        Jd, r0d = to_dev(J, dtype), to_dev(r0, dtype)
        d_ws = torch.zeros(n, dtype=tdt, device=dev)
        d_na = torch.full((n,), float("nan"), dtype=tdt, device=dev)
        st = torch.full((2,), 99, dtype=torch.int32, device=dev)
        work = torch.empty(_lib.gnmppi_ggn_workspace(CODE[dtype], m, n), dtype=torch.uint8, device=dev)
        _lib.gnmppi_ggn_step(Jd, r0d, lam, d_ws, work, st[0:1])
        _lib.gnmppi_ggn_step_noalloc(Jd, r0d, lam, d_na, st[1:2])
        torch.cuda.synchronize()
        assert st.cpu().tolist() == [_lib.OK, _lib.OK]
        np.testing.assert_array_equal(host(d_na), host(d_ws), err_msg=f"m={m} n={n}")
        assert_parity(host(d_na), ggn.direction(J, r0, lam), dtype, f"m={m} n={n}")

