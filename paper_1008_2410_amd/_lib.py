"""ctypes declarations of the C ABI in include/fmm2d.h and include/fmm2d_adaptive.h
(argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm2d.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_ERANGE, FMM_ESTATE = 0, -1, -2, -3, -4, -5
FMM_FP64, FMM_MIXED = 0, 1
FMM_OPT_SCHEDULE, FMM_OPT_COARSE_LEVEL, FMM_OPT_TIMING = 1, 2, 3
FMM_OPT_NEAR_MUTUAL, FMM_OPT_DENSE_LEAF, FMM_OPT_NEAR_OCCUPANCY, FMM_OPT_VALIDATE = 6, 7, 8, 9
FMM_ACC_GAMMA, FMM_ACC_X, FMM_IDENTITY = 1, 2, 4
FMM_T_PACK, FMM_T_FAR, FMM_T_P2P, FMM_T_FINAL, FMM_T_TOTAL, FMM_T_COUNT = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "FMM_OK", -1: "FMM_EINVAL", -2: "FMM_ENOMEM", -3: "FMM_EDEVICE", -4: "FMM_ERANGE",
                -5: "FMM_ESTATE"}

# Every exported symbol with (restype, argtypes).
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
SIGNATURES = {
    "fmm_build_tree": (_I, [_P, _I64, _I, _P, _P, ctypes.POINTER(_P)]),
    "fmm_build_tree_host": (_I, [_P, _I64, _I, _P, _P, ctypes.POINTER(_P)]),
    "fmm_rebuild_tree": (_I, [_P, _P, _I64, _P, _P, ctypes.POINTER(_P)]),
    "fmm_tree_info": (_I, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "fmm_share_workspace": (_I, [_P, _P]),
    "fmm_tree_permutation": (_I, [_P, _P, _P, _P]),
    "fmm_tree_levels": (_I, [_P, _P, _I]),
    "fmm_velocity": (_I, [_P, _P, _D, _I, _I, _P, _P, _P]),
    "fmm_velocity_parts": (_I, [_P, _P, _D, _I, _I, _P, _P, _P, _P]),
    "fmm_velocity_noalloc": (_I, [_P, _P, _D, _I, _I, _P, _P, _P]),
    "fmm_velocity_backward": (_I, [_P, _P, _D, _I, _I, _P, _P, _P, _P, _P, _P, _P]),
    "fmm_transport_step": (_I, [_P, _P, _D, _I, _I, _P, _P, _P, _D, _P]),
    "fmm_transport_vjp": (_I, [_P, _P, _D, _I, _I, _P, _D, _I, _P, _P, _P, _P]),
    "fmm_set_option": (_I, [_P, _I, _I64]),
    "fmm_get_timings": (_I, [_P, _P, _P]),
    "fmm_get_timeline": (_I, [_P, _P, _I]),
    "fmm_near_plan_info": (_I, [_P, _P, _P, _P]),
    "fmm_destroy_tree": (None, [_P]),
    "fmm_last_error": (ctypes.c_char_p, []),
    # include/fmm2d_adaptive.h
    "fmm_atree_build": (_I, [_P, _I64, _I, _I, _P, _P, ctypes.POINTER(_P)]),
    "fmm_atree_build_host": (_I, [_P, _I64, _I, _I, _P, _P, ctypes.POINTER(_P)]),
    "fmm_atree_rebuild": (_I, [_P, _P, _I64, _P, _P, ctypes.POINTER(_P)]),
    "fmm_atree_velocity_backward": (_I, [_P, _P, _D, _I, _I, _P, _P, _P, _P, _P, _P, _P]),
    "fmm_atree_transport_step": (_I, [_P, _P, _D, _I, _I, _P, _P, _P, _D, _P]),
    "fmm_atree_transport_vjp": (_I, [_P, _P, _D, _I, _I, _P, _D, _I, _P, _P, _P, _P]),
    "fmm_atree_info": (_I, [_P, _P, _P]),
    "fmm_atree_share_workspace": (_I, [_P, _P]),
    "fmm_atree_leaves": (_I, [_P, _P, _P, _P]),
    "fmm_atree_velocity": (_I, [_P, _P, _D, _I, _I, _P, _P, _P]),
    "fmm_atree_velocity_parts": (_I, [_P, _P, _D, _I, _I, _P, _P, _P, _P]),
    "fmm_atree_set_option": (_I, [_P, _I, _I64]),
    "fmm_atree_destroy": (None, [_P]),
}
FMM_AT_KEYS = ("cells", "leaves", "u", "v", "w", "x", "deepest", "p2p_pairs")

_lib = None


class FmmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; fails loudly if it has not been built.

    torch is imported first: it ships its own HIP runtime (same soname), and the
    library must bind to that copy rather than bring a second runtime into the process."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1008_2410_amd.build` "
                               "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str):
    if status != FMM_OK:
        msg = load().fmm_last_error().decode(errors="replace")
        raise FmmError(status, where, msg)
