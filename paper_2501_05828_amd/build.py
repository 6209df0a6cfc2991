"""Builds libultraray.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32
instruction selection disabled, then linked into one shared library whose
exported symbols are exactly the C ABI in include/ultraray.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libultraray.so")
SOURCES = ["ur_host.cpp", "bvh.cpp", "scatter_grid.cpp", "k_trace.hip", "k_trace_rays.hip", "k_bin.hip", "k_signal.hip", "k_mlp.hip",
           "k_adjoint.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]
# Per-file additions.  The trace kernels are persistent loops at the
# 128-register limit of 4 waves per SIMD: machine-level loop-invariant code
# motion hoists the materialisation of their 64-bit constants (the FP64
# polynomial coefficients of emission and acos: two moves each) out of the
# loop, where they no longer fit and spill to scratch, so that every use waits
# on a scratch load.  Without that pass the extend kernel needs 111 registers
# and no scratch, and runs about a tenth faster.  The explicit-ray kernel
# (k_trace_rays.hip, the event-log path) is built without loop unrolling as
# well: with it, a call with many rays lost some direct-hit records.  The
# adjoint's replay kernel, held to 256 registers, spills less without the
# pass (all gradients of the large scene: 2.62 s with it, 2.08 s without).
EXTRA = {"k_trace.hip": ["-mllvm", "-disable-machine-licm"],
         "k_trace_rays.hip": ["-mllvm", "-disable-machine-licm", "-fno-unroll-loops"],
         "k_adjoint.hip": ["-mllvm", "-disable-machine-licm"]}


def flags_for(src: str) -> list:
    """hipcc flags of one translation unit."""
    return [*FLAGS, *EXTRA.get(src, [])]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC, *lang, *flags_for(src), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
