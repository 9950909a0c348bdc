"""Build libgnmppi.so for gfx950 with hipcc, in-tree.

Usage: python -m paper_2512_04579_amd.build  (or call ``build()``).
Every HIP source is compiled to an object in parallel, then linked into a
shared library next to this file.  Always compiles (no up-to-date check).
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(HERE, "libgnmppi.so")
ARCH = "gfx950"

# Longest compiles first (the sweep units instantiate one kernel per 16-row
# class), so the parallel build ends with the short ones.
SOURCES = ["sweep_batch_inv.hip", "sweep_batch_dir.hip", "sweep_f32.hip", "sweep_f64.hip",
           "fused.hip", "dense.hip", "gemm.hip", "gemm_plain.hip", "rollout.hip", "abi.cpp",
           "batch.cpp", "sample.hip", "mppi.hip", "mlp.hip"]

# Packed FP32 VALU ops are switched off for every HIP translation unit.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# The sweep units keep their f64 MFMA accumulators in ordinary VGPRs: the
# update waves select between tiles and zero pivot rows in place, which with
# accumulators in AGPRs costs a copy out and back for every tile (measured: the
# sweep 11 % faster, no spills).  So does the plain-BF16 contraction unit
# (measured 0.8 % faster for the whole c4 iteration), while the BF16x3
# contraction keeps AGPRs (with VGPRs c2 was no faster).
EXTRA_FLAGS = {src: ["-mllvm", "-amdgpu-mfma-vgpr-form"]
               for src in ("sweep_batch_inv.hip", "sweep_batch_dir.hip", "sweep_f32.hip",
                           "sweep_f64.hip", "gemm_plain.hip")}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [_hipcc(), *HIPCC_FLAGS, *EXTRA_FLAGS.get(src, []), f"-I{INCLUDE}", f"-I{CSRC}", *lang,
           "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
