"""ctypes declarations of libsf.so (the C ABI in include/sf.h).

The shared library is built in-tree by paper_1801_04720_amd/build.py.  There is
no fallback of any kind: if the library is missing or fails to load, every
call raises.
"""
from __future__ import annotations

import ctypes as ct
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SF_LIB_PATH") or os.path.join(_PKG, "libsf.so")

SF_OK, SF_EINVAL, SF_EUNSUPPORTED, SF_EHIP, SF_ENOMEM = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "SF_OK", 1: "SF_EINVAL", 2: "SF_EUNSUPPORTED", 3: "SF_EHIP", 4: "SF_ENOMEM"}

P = ct.c_void_p
I = ct.c_int
U32 = ct.c_uint32
F = ct.c_float
SZ = ct.c_size_t


class SfCamera(ct.Structure):
    _fields_ = [("f", ct.c_float), ("B", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float)]


class SfPair(ct.Structure):
    _fields_ = [("H", ct.c_int), ("W", ct.c_int), ("D", ct.c_int), ("pitch", ct.c_int),
                ("left", ct.c_void_p), ("right", ct.c_void_p), ("wta", ct.c_void_p),
                ("disp", ct.c_void_p), ("valid", ct.c_void_p)]


class SfAggTuning(ct.Structure):
    _fields_ = [("chains_per_block", ct.c_int), ("prefetch", ct.c_int), ("order", ct.c_int),
                ("persistent_per_cu", ct.c_int), ("packed", ct.c_int)]


class SfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


# name -> (restype, argtypes)
SIGNATURES = {
    "sf_abi_version": (I, []),
    "sf_last_error": (ct.c_char_p, []),
    "sf_census": (I, [P, I, I, I, P, P]),
    "sf_cost": (I, [P, P, I, I, I, I, P, P]),
    "sf_sgm_workspace_bytes": (SZ, [I, I, I]),
    "sf_sgm_aggregate": (I, [P, I, I, I, I, I, U32, P, P, SZ, P]),
    "sf_sgm_set_epilogue": (I, [I]),
    "sf_sgm_aggregate_census": (I, [P, P, I, I, I, I, I, I, U32, P, P, SZ, P]),
    "sf_debug_checked": (I, []),
    "sf_debug_check": (I, [ct.POINTER(ct.c_uint32), I]),
    "sf_debug_selftest": (I, [I, P]),
    "sf_wta_lr": (I, [P, P, P, I, I, I, I, I, I, P, P, P, P, P, P]),
    "sf_combine": (I, [P, P, P, P, P, I, I, ct.POINTER(SfCamera), P, P, P, P, P]),
    "sf_plan_workspace_bytes": (SZ, [P]),
    "sf_plan_destroy": (I, [P]),
    "sf_frame_plan_create": (I, [I, I, I, I, I, I, I, ct.POINTER(SfAggTuning), ct.POINTER(P)]),
    "sf_frame_run": (I, [P, P, P, P, P, I, P, ct.POINTER(SfCamera), P, P, P, P, P, P, P, P, P, SZ,
                         P]),
    "sf_lrnet_nparams": (I, []),
    "sf_lrnet_workspace_bytes": (SZ, [I, I, I, I]),
    "sf_lrnet_forward": (I, [P, P, I, I, I, P, P, SZ, P]),
    "sf_lrnet_mask": (I, [P, P, P, I, I, P, P, P]),
    "sf_lrnet_grad": (I, [P, P, P, I, I, I, P, P, P, SZ, P]),
    "sf_lrnet_backward": (I, [P, P, P, I, I, I, P, P, SZ, P]),
    "sf_lrnet_forward_noalloc": (I, [P, P, I, I, I, P, P]),
    "sf_mask_agreement": (I, [P, P, I, P, P]),
    "sf_lrnet_adam": (I, [P, P, P, P, I, F, F, F, F, F, F, P]),
    "sf_frame_run_learned": (I, [P, P, P, P, P, I, P, ct.POINTER(SfCamera), P, P, P, P, P, P, P, P,
                                 P, P, SZ, P]),
    "sf_batch_plan_create": (I, [ct.POINTER(SfPair), I, I, I, I, ct.POINTER(SfAggTuning), I, SZ,
                                 ct.POINTER(P)]),
    "sf_batch_plan_info": (I, [P, ct.POINTER(I), ct.POINTER(I)]),
    "sf_batch_run": (I, [P, P, SZ, P]),
    "sf_batch_capture": (I, [P, P, SZ, P]),
    "sf_batch_launch": (I, [P, P]),
    "sf_agg_autotune": (I, [I, I, I, I, I, I, P, ct.POINTER(SfAggTuning), ct.POINTER(F)]),
    "sf_frame_autotune": (I, [I, I, I, I, I, I, I, P, ct.POINTER(SfAggTuning), ct.POINTER(F)]),
    "sf_prof_enable": (I, [I]),
    "sf_prof_only": (I, [ct.c_char_p]),
    "sf_prof_disable": (I, []),
    "sf_prof_query": (I, [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(I)]),
    "sf_sgm_aggregate_adaptive": (I, [P, P, I, I, I, I, I, I, U32, P, P, SZ, P]),
    "sf_wta_right_diag": (I, [P, I, I, I, P, P]),
    "sf_lr_check": (I, [P, P, P, I, I, I, P, P, P]),
    "sf_median3x3": (I, [P, P, I, I, P, P]),
    "sf_densify_workspace_bytes": (SZ, [I]),
    "sf_densify": (I, [P, P, I, I, P, P, P, SZ, P]),
    "sf_temporal_check": (I, [P, P, P, P, I, I, F, F, P, P]),
    "sf_flow_workspace_bytes": (SZ, [I, I, I]),
    "sf_flow": (I, [P, P, I, I, I, I, I, I, I, ct.c_uint64, I, P, P, P, P, SZ, P]),
    "sf_probe_stream": (I, [P, P, SZ, I, P]),
    "sf_probe_pk_u16": (I, [P, I, I, P]),
}

_lib = None


def lib() -> ct.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run paper_1801_04720_amd/build.py (hipcc, gfx950)")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != SF_OK:
        msg = lib().sf_last_error().decode(errors="replace")
        raise SfError(status, msg)
