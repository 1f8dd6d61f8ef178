"""Build libgcp.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1906_01687_amd.build``.  Objects go to ``_build/`` at
the repository root; the shared library lands next to this file.
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
OUT = os.path.join(HERE, "libgcp.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["abi.cpp", "sample.hip", "grad.hip", "adam.hip", "batched.hip"]
# the kernels of each mode count d = 1..8 are instantiated in their own object
MODE_COUNTS = range(1, 9)
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
    # packed FP32 instructions stay off: some of their forms have given wrong
    # results on this target now and then, so the compiler may not emit them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _compile(job) -> str:
    src, defines = job if isinstance(job, tuple) else (job, {})
    stem = os.path.splitext(src)[0] + "".join(f"_{k.lower()}{v}" for k, v in defines.items())
    obj = os.path.join(BUILD_DIR, stem + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{k}={v}" for k, v in defines.items()], "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = [("inst.hip", {"GCP_INST_D": d}) for d in MODE_COUNTS] + list(SOURCES)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
