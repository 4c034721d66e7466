"""Builds libdsfft.so (HIP, gfx950) in-tree from csrc/.

Usage: python -m paper_2604_00567_amd.build   (or build() from Python)

Every HIP translation unit is compiled with hipcc for gfx950 with FP
contraction off (only the explicit FMAs of the butterfly are fused), denormals
kept, and packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdsfft.so")

HIP_SOURCES = ["api.cpp", "batch.cpp", "serve.cpp", "serve_loop.cpp", "tune.cpp", "scratch.cpp", "kernels_f16.hip", "kernels_f32.hip",
               "kernels_f16f32.hip", "kernels_batch.hip"]
CXX_SOURCES = ["tables.cpp"]

ARCH = os.environ.get("DSFFT_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-fno-gpu-flush-denormals-to-zero",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    if src in HIP_SOURCES:
        cmd = [_hipcc(), "-x", "hip"] + COMMON + HIP_FLAGS + ["-c", path, "-o", obj]
    else:
        cmd = [_hipcc()] + COMMON + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = HIP_SOURCES + CXX_SOURCES
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
