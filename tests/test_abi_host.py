"""Host-only checks of the C ABI (no GPU needed).

* the built library loads and exports every function ``include/gnmppi.h``
  declares, and the binding declares a signature for each;
* the ctypes mirror of ``gnmppi_problem`` has the layout a C compiler gives
  the header's struct (checked with gcc);
* invalid arguments are rejected synchronously with GNMPPI_EINVAL /
  GNMPPI_ENOSPACE before anything touches a device;
* workspace queries are pure host arithmetic.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2512_04579_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gnmppi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gnmppi_\w+)\s*\(", text)))


def test_header_declares_the_four_hot_path_calls():
    names = _declared_functions()
    for required in ("gnmppi_rollout", "gnmppi_mppi_update", "gnmppi_reconstruct_jacobian",
                     "gnmppi_ggn_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks a signature for {name}"


def test_problem_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "gnmppi.h"\n'
        "int main(void){printf(\"%zu\", sizeof(gnmppi_problem));\n"
        + "".join(f'printf(" %zu", offsetof(gnmppi_problem, {f}));\n'
                  for f, _ in _lib.GnmppiProblem._fields_)
        + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                   check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(_lib.GnmppiProblem)
    for (name, _), off in zip(_lib.GnmppiProblem._fields_, out[1:]):
        assert getattr(_lib.GnmppiProblem, name).offset == off, name


def test_header_compiles_as_c_and_cxx(tmp_path):
    src = tmp_path / "use.c"
    src.write_text('#include "gnmppi.h"\nint f(void){return GNMPPI_EINVAL;}\n')
    for cmd in (["gcc", "-std=c99", "-Wall", "-Werror"], ["g++", "-x", "c++", "-Wall", "-Werror"]):
        subprocess.run(cmd + [f"-I{os.path.join(ROOT, 'include')}", "-c", str(src), "-o",
                              str(tmp_path / "use.o")], check=True)


def _problem(**kw):
    base = dict(model=_lib.MODEL_CHAIN, dtype=_lib.F32, nx=64, nu=2, N=50, n_masses=16, dt=0.05,
                k_lin=1.0, k_cub=0.5, mass=1.0, q=0x1000, r=0x2000, x_ref=0x3000)
    base.update(kw)
    return _lib.GnmppiProblem(**base)


@pytest.mark.parametrize("kw", [
    dict(n_masses=17, nx=68), dict(nx=63), dict(nu=3), dict(N=0), dict(dt=0.0), dict(mass=0.0),
    dict(dtype=7), dict(q=None), dict(model=9),
    dict(model=_lib.MODEL_DOUBLE_INTEGRATOR, nx=10, nu=5),
])
def test_rollout_rejects_bad_problems(kw):
    lib = _lib.load()
    p = _problem(**kw)
    rc = lib.gnmppi_rollout(ctypes.byref(p), 0x10, 0x20, 0x30, 4096, 4096, 0x40, 4096, 0x50, None,
                            None, None)
    assert rc == _lib.EINVAL


def test_rollout_rejects_bad_sizes():
    lib = _lib.load()
    p = _problem()
    args = lambda K, ldw, ldr, C=0x50, c0=None, r0=None, R=0x40: (  # noqa: E731
        ctypes.byref(p), 0x10, 0x20, 0x30, ldw, K, R, ldr, C, r0, c0, None)
    assert lib.gnmppi_rollout(*args(4096, 4095, 4096)) == _lib.EINVAL   # ldw < K
    assert lib.gnmppi_rollout(*args(4096, 4096, 100)) == _lib.EINVAL    # ldr < K
    assert lib.gnmppi_rollout(*args(-1, 4096, 4096)) == _lib.EINVAL
    assert lib.gnmppi_rollout(*args(0, 0, 0)) == _lib.EINVAL            # nothing to roll out
    assert lib.gnmppi_rollout(*args(8, 8, 8, C=None, R=None)) == _lib.EINVAL  # neither R nor C
    assert lib.gnmppi_rollout(*args(8, 8, 8, r0=0x60)) == _lib.EINVAL   # r0 without c0


def test_other_entry_points_reject_bad_arguments():
    lib = _lib.load()
    assert lib.gnmppi_sample(_lib.F32, 0, 8, 1.0, 1, 0, 1, 0x10, 8, None) == _lib.EINVAL
    assert lib.gnmppi_sample(_lib.F32, 4, 7, 1.0, 1, 0, 1, 0x10, 8, None) == _lib.EINVAL  # odd K
    assert lib.gnmppi_sample(_lib.F32, 4, 8, 1.0, 1, 0, 1, 0x10, 7, None) == _lib.EINVAL
    assert lib.gnmppi_sample(3, 4, 8, 1.0, 1, 0, 1, 0x10, 8, None) == _lib.EINVAL
    assert lib.gnmppi_mppi_update(_lib.F32, 4, 8, 0x10, 0x20, 8, 0.0, 0x30, None, None, None) == _lib.EINVAL
    assert lib.gnmppi_mppi_update(_lib.F32, 4, 20000, 0x10, 0x20, 20000, 1.0, 0x30, None, None, None) == _lib.EINVAL
    ws = lib.gnmppi_jacobian_workspace(_lib.F32, 3300, 100, 4096)
    assert ws > 0
    # n beyond the LDS-resident limit, misaligned or short workspace
    assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 300, 193, 512, 0x100, 512, 0x200, 0x300, 512,
                                           0, 0.0, 0x400, 193, 0x1000, 1 << 30, None, None) == _lib.EINVAL
    assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                           0, 0.0, 0x400, 100, 0x1008, ws, None, None) == _lib.EINVAL
    assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                           0, 0.0, 0x400, 100, 0x1000, ws - 1, None, None) == _lib.ENOSPACE
    assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                           1, 0.0, 0x400, 100, 0x1000, ws, None, None) == _lib.EINVAL  # MC, sigma2=0
    assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                           1 | _lib.JAC_GRAM_READY, 0.1, 0x400, 100, 0x1000, ws, None,
                                           None) == _lib.EINVAL  # gram flag only for LS
    # the two-phase flags need LS + GRAM_READY and exclude each other; unknown bits are rejected
    for method in (_lib.JAC_S_ONLY, _lib.JAC_APPLY_ONLY,
                   _lib.JAC_GRAM_READY | _lib.JAC_S_ONLY | _lib.JAC_APPLY_ONLY,
                   _lib.JAC_MC | _lib.JAC_GRAM_READY | _lib.JAC_S_ONLY, 0x2000):
        assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                               method, 0.1, 0x400, 100, 0x1000, ws, None, None) == _lib.EINVAL
    wsd = lib.gnmppi_jacobian_workspace(_lib.F64, 3300, 100, 4096)
    assert lib.gnmppi_reconstruct_jacobian(_lib.F64, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                           _lib.JAC_BF16, 0.0, 0x400, 100, 0x1000, wsd, None, None) == _lib.EINVAL
    assert lib.gnmppi_reconstruct_jacobian(_lib.F32, 3300, 100, 4096, 0x100, 4096, 0x200, 0x300, 4096,
                                           _lib.JAC_BF16 | _lib.JAC_BF16X3, 0.0, 0x400, 100, 0x1000, ws,
                                           None, None) == _lib.EINVAL
    assert lib.gnmppi_perturbation_gram(_lib.F32, 3300, 100, 4096, 0x300, 4095, 0x1000, ws, None, None) == _lib.EINVAL
    assert lib.gnmppi_perturbation_gram(_lib.F32, 3300, 100, 4096, 0x300, 4096, 0x1000, ws - 1, None, None) == _lib.ENOSPACE
    wg = lib.gnmppi_ggn_workspace(_lib.F64, 120, 40)
    assert wg > 0
    assert lib.gnmppi_ggn_step(_lib.F64, 120, 40, 0x100, 39, 0x200, 1, 0.0, 0x300, 0x1000, wg, None, None) == _lib.EINVAL
    assert lib.gnmppi_ggn_step(_lib.F64, 120, 40, 0x100, 40, 0x200, 1, -1.0, 0x300, 0x1000, wg, None, None) == _lib.EINVAL
    assert lib.gnmppi_ggn_step(_lib.F64, 120, 40, 0x100, 40, 0x200, 1, 0.0, 0x300, 0x1000, wg - 8, None, None) == _lib.ENOSPACE
    p = _problem()
    assert lib.gnmppi_line_search(ctypes.byref(p), 0x10, 0x20, 0x30, 0x40, 0, None, None, None,
                                  None) == _lib.EINVAL
    assert lib.gnmppi_line_search(ctypes.byref(p), 0x10, 0x20, 0x30, 0x40, 65, None, None, None,
                                  None) == _lib.EINVAL
    assert lib.gnmppi_sigma_points(_lib.F64, 4, 1.0, 0x10, 7, None) == _lib.EINVAL


def test_status_strings_and_version():
    assert _lib.status_string(_lib.ENOTPD) == "normal matrix not positive definite"
    assert _lib.status_string(123) == "unknown status"
    assert _lib.gnmppi_abi_version() == 4


def test_mlp_entry_points_reject_bad_arguments():
    lib = _lib.load()
    assert lib.gnmppi_mlp_param_count(64, 256, 100) == 256 * 64 + 256 + 256 * 256 + 256 + 100 * 256 + 100
    assert lib.gnmppi_mlp_param_count(0, 256, 100) == 0
    ws = lib.gnmppi_mlp_workspace(64, 256, 100, 1024)
    assert ws == (6 * 1024 * 256 + 2 * 1024 * 100) * 4
    assert lib.gnmppi_mlp_workspace(64, 256, 100, 0) == 0
    assert lib.gnmppi_mlp_forward(64, 256, 100, 1024, 0x100, 0x200, 0x300, 0x1000, ws - 4, None) == _lib.ENOSPACE
    assert lib.gnmppi_mlp_forward(64, 256, 100, 1024, 0x100, 0x200, 0x300, 0x1008, ws, None) == _lib.EINVAL
    assert lib.gnmppi_mlp_forward(64, 5000, 100, 1024, 0x100, 0x200, 0x300, 0x1000, ws, None) == _lib.EINVAL
    assert lib.gnmppi_mlp_backward(64, 256, 100, 1024, 0x100, 0x200, None, None, 0x400, 0x1000, ws,
                                   None) == _lib.EINVAL
    assert lib.gnmppi_mlp_adam(10, 0x10, 0x20, 0x30, 0x40, 0x50, 1e-3, 0.9, 0.999, 1e-8, 0, None) == _lib.EINVAL
    assert lib.gnmppi_mlp_adam(10, 0x10, 0x20, 0x30, 0x40, 0x50, 1e-3, 1.0, 0.999, 1e-8, 1, None) == _lib.EINVAL


def test_sample_rollout_rejects_bad_arguments():
    lib = _lib.load()
    p = _problem()
    K = 64

    def call(W=0x30, ldw=K, K=K, anti=1, sigma=0.3, R=0x40, C=None, r0=None, c0=None, U=0x20):
        return lib.gnmppi_sample_rollout(ctypes.byref(p), 0x10, U, sigma, 1, 0, anti, W, ldw, K, R,
                                         K, C, r0, c0, None)

    assert call(W=None) == _lib.EINVAL          # W is the sampler's output
    assert call(U=None) == _lib.EINVAL
    assert call(ldw=K - 1) == _lib.EINVAL
    assert call(K=63, ldw=64) == _lib.EINVAL    # antithetic pairs need even K
    assert call(K=0) == _lib.EINVAL
    assert call(sigma=float("nan")) == _lib.EINVAL
    assert call(R=None, C=None) == _lib.EINVAL  # nothing wanted of the K columns
    assert call(r0=0x50, c0=None) == _lib.EINVAL


def test_line_search_nominal_rejects_bad_arguments():
    lib = _lib.load()
    p = _problem()

    def call(L=16, Rc=0x50, r0=0x60, c0=0x70, U=0x20):
        return lib.gnmppi_line_search_nominal(ctypes.byref(p), 0x10, U, 0x30, 0x40, L, None, None,
                                              None, Rc, r0, c0, None)

    assert call(Rc=None) == _lib.EINVAL   # the candidates' residuals have nowhere to go
    assert call(r0=None) == _lib.EINVAL
    assert call(c0=None) == _lib.EINVAL
    assert call(U=None) == _lib.EINVAL
    assert call(L=0) == _lib.EINVAL
    assert call(L=65) == _lib.EINVAL


def test_ggn_direction_rejects_bad_arguments():
    lib = _lib.load()
    LS_READY = _lib.JAC_LS | _lib.JAC_GRAM_READY
    ws = lib.gnmppi_ggn_direction_workspace(_lib.F32, 3300, 100, 4096)
    # the Jacobian workspace followed by the GGN workspace
    assert ws == lib.gnmppi_jacobian_workspace(_lib.F32, 3300, 100, 4096) + \
        lib.gnmppi_ggn_workspace(_lib.F32, 3300, 100)
    assert lib.gnmppi_ggn_direction_workspace(_lib.F32, 0, 100, 4096) == 0

    def call(method, dtype=_lib.F32, n=100, sigma2=0.1, lam=0.0, work=0x1000, wbytes=ws, ldr=4096):
        return lib.gnmppi_ggn_direction(dtype, 3300, n, 4096, 0x100, ldr, 0x200, 0x300, 4096, method,
                                        sigma2, lam, 0x400, work, wbytes, None, None)

    for method in (_lib.JAC_MC | _lib.JAC_GRAM_READY, _lib.JAC_MC | _lib.JAC_S_ONLY,
                   LS_READY | _lib.JAC_S_ONLY | _lib.JAC_APPLY_ONLY,
                   LS_READY | _lib.JAC_BF16 | _lib.JAC_BF16X3, LS_READY | 0x2000, 2):
        assert call(method) == _lib.EINVAL
    assert call(_lib.JAC_MC, sigma2=0.0) == _lib.EINVAL
    assert call(LS_READY, lam=-1.0) == _lib.EINVAL
    assert call(LS_READY, lam=float("inf")) == _lib.EINVAL
    assert call(LS_READY, n=193) == _lib.EINVAL
    assert call(LS_READY, ldr=4095) == _lib.EINVAL
    assert call(LS_READY, work=0x1008) == _lib.EINVAL
    assert call(LS_READY, wbytes=ws - 1) == _lib.ENOSPACE
    wsd = lib.gnmppi_ggn_direction_workspace(_lib.F64, 3300, 100, 4096)
    assert call(LS_READY | _lib.JAC_BF16X3, dtype=_lib.F64, wbytes=wsd) == _lib.EINVAL


def test_noalloc_ggn_step_rejects_without_touching_a_device():
    lib = _lib.load()
    # gnmppi_ggn_workspace(F32, 6913, 192) exceeds the 8 MiB scratch
    assert _lib.gnmppi_ggn_workspace(_lib.F32, 6913, 192) > 8 << 20
    assert _lib.gnmppi_ggn_workspace(_lib.F32, 6912, 192) <= 8 << 20
    args = (0x1000, 192, 0x2000, 1, 0.0, 0x3000, None, None)
    assert lib.gnmppi_ggn_step_noalloc(_lib.F32, 6913, 192, *args) == _lib.ENOSPACE
    assert lib.gnmppi_ggn_step_noalloc(_lib.F32, 6913, 193, *args) == _lib.EINVAL
    assert lib.gnmppi_ggn_step_noalloc(_lib.F32, 100, 50, None, 50, 0x2000, 1, 0.0, 0x3000, None,
                                       None) == _lib.EINVAL
