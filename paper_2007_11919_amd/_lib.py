"""ctypes loader for libmds.so: symbol signatures only, no logic."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmds.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
P_i64 = ctypes.POINTER(c_i64)
P_i32 = ctypes.POINTER(c_i32)
P_dbl = ctypes.POINTER(c_dbl)


class ServeStats(ctypes.Structure):
    _fields_ = [(name, c_i64) for name in (
        "submitted", "admitted", "completed", "queued", "in_flight", "steps",
        "tiles", "points", "bytes_in_use", "budget_bytes")]


SIGNATURES = {
    "mds_sample_landmarks": (c_i32, [c_i64, c_i64, c_u64, P_i64]),
    "mds_fit_landmarks": (c_i32, [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i32, c_u64,
                                  P_i64, c_vp, ctypes.POINTER(c_vp)]),
    "mds_embed": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "mds_free": (None, [c_vp]),
    "mds_fit_from_sqdist": (c_i32, [c_vp, c_i64, c_i64, c_i32, c_vp, ctypes.POINTER(c_vp)]),
    "mds_embed_from_sqdist": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "mds_maxmin_landmarks": (c_i32, [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i64, P_i64, c_vp]),
    "mds_maxmin_landmarks_noalloc": (c_i32, [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i64, P_i64, c_vp]),
    "mds_pivot_mds": (c_i32, [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i32, c_u64, P_i64, c_vp, c_i64,
                              P_dbl, P_i32, c_vp]),
    "mds_embed_affine": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "mds_divide_conquer": (c_i32, [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i64, c_i32, c_u64,
                                   c_vp, c_i64, P_dbl, P_i32, c_vp, c_vp]),
    "mds_model_info": (c_i32, [c_vp, P_i64, P_i64, P_i64, P_i32, P_i32]),
    "mds_get_landmarks": (c_i32, [c_vp, P_i64]),
    "mds_get_eigenvalues": (c_i32, [c_vp, P_dbl]),
    "mds_get_landmark_coords": (c_i32, [c_vp, P_dbl]),
    "mds_get_q": (c_i32, [c_vp, P_dbl]),
    "mds_model_bytes": (c_i64, [c_vp]),
    "mds_fit_stats": (c_i32, [c_vp, P_i32, P_i32]),
    "mds_last_error": (ctypes.c_char_p, []),
    "mds_last_hip_error": (c_i32, []),
    "mds_serve_create": (c_i32, [c_i64, c_i32, c_i32, ctypes.POINTER(c_vp)]),
    "mds_serve_add_model": (c_i32, [c_vp, c_vp, P_i32]),
    "mds_serve_submit": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_i64, c_i64, c_i32, c_vp, c_i64, P_i64]),
    "mds_serve_poll": (c_i32, [c_vp, c_i64, P_i32, P_dbl, P_dbl, P_dbl]),
    "mds_serve_wait": (c_i32, [c_vp, c_i64, c_dbl]),
    "mds_serve_stats": (c_i32, [c_vp, ctypes.POINTER(ServeStats)]),
    "mds_serve_now": (c_dbl, [c_vp]),
    "mds_serve_destroy": (None, [c_vp]),
    "mds_debug_bounded": (c_u64, [c_u64, c_u64, c_i32, ctypes.POINTER(c_u64)]),
}

_LIB = None


def lib():
    """Load libmds.so (built in-tree by paper_2007_11919_amd.build)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_2007_11919_amd.build.build(); "
                "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB
