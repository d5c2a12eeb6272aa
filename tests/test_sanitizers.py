"""CPU code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

* The oracle (test infrastructure) built with both sanitizers and its pins run against it
  (ORACLE_SANITIZE=1, gcc's libasan preloaded into the test process).
* The library's host tree build (host_tree.cpp, the reference the device build is checked
  against) built with both sanitizers into a driver that checks every array against its
  definition on seeded and degenerate inputs (tests/sanitize_host_tree.cpp).
* The C ABI's argument checks, status codes and error messages in a build of libfmm2d.so
  whose host code carries both sanitizers (device code unchanged), called through ctypes
  before any device work.
Each runs in a child process so that a sanitizer report ends that process and fails the
test with its output.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env_extra=None, timeout=600):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra or {})
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    return out


def _gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()


def test_oracle_pins_under_sanitizers():
    import oracle
    env = {"ORACLE_SANITIZE": "1", "LD_PRELOAD": _gcc_runtime("libasan.so")}
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT, check=True,
                   env={**os.environ, "ORACLE_SANITIZE": "1"})
    out = _run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "tests/test_oracle_adaptive.py",
                "tests/test_cost_model.py", "-x", "-q", "-p", "no:cacheprovider"], env)
    assert " passed" in out
    assert oracle.SANITIZE is False  # this process keeps the plain build


def test_host_tree_build_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_tree_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "tests/sanitize_host_tree.cpp",
                    "paper_1008_2410_amd/csrc/host_tree.cpp", "-o", exe], cwd=ROOT, check=True)
    out = _run([exe])
    assert "host tree checks passed" in out


ABI_SCRIPT = r"""
import ctypes, sys
from paper_1008_2410_amd import _lib as L
lib = ctypes.CDLL(sys.argv[1])
for name, (res, args) in L.SIGNATURES.items():
    fn = getattr(lib, name)
    fn.restype, fn.argtypes = res, args
h = ctypes.c_void_p()
xy = ctypes.c_void_p(0x1000)  # never dereferenced: the checks come first
P = None
assert lib.fmm_build_tree(P, 10, 4, P, P, ctypes.byref(h)) == L.FMM_EINVAL and b"xy" in lib.fmm_last_error()
assert lib.fmm_build_tree(xy, 0, 4, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_build_tree(xy, 10, 0, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_build_tree(xy, 10, 13, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_build_tree(xy, 1 << 31, 4, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_build_tree(xy, 10, 4, P, P, P) == L.FMM_EINVAL
bad_root = (ctypes.c_double * 3)(0.0, 0.0, -1.0)
assert lib.fmm_build_tree(xy, 10, 4, bad_root, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_build_tree_host(P, 10, 4, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_rebuild_tree(P, xy, 10, P, P, ctypes.byref(h)) == L.FMM_ESTATE
assert lib.fmm_velocity(P, xy, 0.1, 8, 0, P, P, xy) == L.FMM_ESTATE
assert lib.fmm_velocity(P, xy, 0.1, 8, 0, P, P, P) == L.FMM_EINVAL
assert lib.fmm_velocity_noalloc(P, xy, 0.1, 8, 0, P, P, xy) == L.FMM_ESTATE
assert lib.fmm_velocity_parts(P, xy, 0.1, 8, 0, P, P, P, xy) == L.FMM_EINVAL
assert lib.fmm_velocity_backward(P, xy, 0.1, 8, 0, xy, P, P, xy, P, P, P) == L.FMM_ESTATE
assert lib.fmm_transport_step(P, xy, 0.1, 8, 0, P, P, P, 0.1, xy) == L.FMM_EINVAL
assert lib.fmm_transport_step(P, xy, 0.1, 8, 0, P, P, xy, float("inf"), xy) == L.FMM_EINVAL
assert lib.fmm_transport_vjp(P, xy, 0.1, 8, 0, xy, 0.1, 8, P, P, xy, xy) == L.FMM_EINVAL
assert lib.fmm_transport_vjp(P, xy, 0.1, 8, 0, P, 0.1, 0, P, P, xy, xy) == L.FMM_EINVAL
assert lib.fmm_share_workspace(P, P) == L.FMM_ESTATE
assert lib.fmm_set_option(P, 1, 0) == L.FMM_ESTATE
assert lib.fmm_tree_info(P, P, P, P, P, P, P, P) == L.FMM_ESTATE
assert lib.fmm_tree_levels(P, P, 4) == L.FMM_ESTATE
assert lib.fmm_tree_permutation(P, xy, P, P) == L.FMM_ESTATE
assert lib.fmm_near_plan_info(P, P, P, P) == L.FMM_ESTATE
assert lib.fmm_get_timings(P, P, P) == L.FMM_ESTATE
assert lib.fmm_get_timeline(P, P, 8) == L.FMM_ESTATE
lib.fmm_destroy_tree(P)
assert lib.fmm_atree_build(P, 10, 16, 6, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_atree_build(xy, 10, 0, 6, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_atree_build(xy, 10, 16, 16, P, P, ctypes.byref(h)) == L.FMM_EINVAL
assert lib.fmm_atree_set_option(P, L.FMM_OPT_NEAR_OCCUPANCY, 5) == L.FMM_ESTATE
assert lib.fmm_atree_velocity(P, xy, 0.1, 8, 0, P, P, P) == L.FMM_EINVAL
assert lib.fmm_atree_transport_vjp(P, xy, 0.1, 8, 0, xy, 0.1, 8, P, P, xy, xy) == L.FMM_EINVAL
assert lib.fmm_atree_share_workspace(P, P) == L.FMM_ESTATE
lib.fmm_atree_destroy(P)
print("abi checks passed")
"""


def test_abi_argument_checks_under_sanitizers(tmp_path):
    from paper_1008_2410_amd import build
    if not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    lib = build.build_library(lib=str(tmp_path / "libfmm2d_san.so"), build_dir=str(tmp_path / "obj"),
                              host_sanitize=True)
    clang = "/opt/rocm/llvm/bin/clang"
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    assert os.path.exists(rt), rt
    out = _run([sys.executable, "-c", ABI_SCRIPT, lib], {"LD_PRELOAD": rt, "PYTHONPATH": ROOT})
    assert "abi checks passed" in out
