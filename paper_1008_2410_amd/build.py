"""Build libfmm2d.so (the gfx950 HIP library) in place with hipcc.

Usage: python -m paper_1008_2410_amd.build
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmm2d.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "tree_build.hip", "adaptive.hip", "adaptive_build.hip", "tables.cpp", "api.cpp",
           "adaptive.cpp"]
ARCH = "gfx950"

# Packed FP32 arithmetic is switched off for the device code (the compiler would
# otherwise form v_pk_* FP32 instructions from scalar float code).
# Code object v5 is accepted by both the system HIP runtime and the one bundled with torch.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mcode-object-version=5"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
           "-Wall", "-Wno-unused-function", *DEVICE_FLAGS, *extra, os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build_library(extra: list[str] | None = None, verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libfmm2d.so; always rebuilds."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    extra = list(extra or [])
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-mcode-object-version=5", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build_library(sys.argv[1:], verbose=True)
