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
           "adaptive.cpp", "host_tree.cpp"]
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


# A build whose host code runs under AddressSanitizer and UndefinedBehaviorSanitizer (device
# code unchanged): each -fsanitize= applies to the host compilation only.
HOST_SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def _compile(src: str, extra: list[str], build_dir: str = BUILD_DIR) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
           "-Wall", "-Wno-unused-function", *DEVICE_FLAGS, *extra, os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build_library(extra: list[str] | None = None, verbose: bool = False, lib: str = LIB,
                  build_dir: str = BUILD_DIR, host_sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link the library (libfmm2d.so in place by
    default); always rebuilds.  host_sanitize: the host code under the sanitizers (a test
    build, loaded with gcc's libasan preloaded)."""
    os.makedirs(build_dir, exist_ok=True)
    extra = list(extra or []) + (HOST_SANITIZE_FLAGS if host_sanitize else [])
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra, build_dir), SOURCES))
    tmp = lib + ".tmp"
    link_extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
                  "-shared-libsan"] if host_sanitize else []
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-mcode-object-version=5", "-shared", "-fPIC", *link_extra, *objs,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build_library(sys.argv[1:], verbose=True)
