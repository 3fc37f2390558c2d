"""ctypes binding of libpbh (include/pbh.h): argument marshalling only.

Every step of the distant-force path runs in the library's HIP kernels; this
module passes device pointers of torch tensors and torch's current HIP stream.
It raises if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbh.so")

PBH_OK = 0
PBH_E_ARG = 1
PBH_E_OOM = 2
PBH_E_HIP = 3
PBH_E_NONFINITE = 4
PBH_E_NBR_OVERFLOW = 5
PBH_E_STATE = 6
PBH_E_INTERNAL = 7
PBH_FP64 = 0
PBH_MIXED = 1
PBH_NOALLOC_MAX_N = 1 << 20

EXPORTS = ("pbh_create", "pbh_destroy", "pbh_set_params", "pbh_get_params", "pbh_build",
           "pbh_force", "pbh_force_buffered", "pbh_build_batched", "pbh_force_batched",
           "pbh_force_batched_buffered", "pbh_irregular",
           "pbh_irregular_batched", "pbh_irregular_noalloc", "pbh_core", "pbh_hermite", "pbh_p3t",
           "pbh_kdk_graph",
           "pbh_kdk_eager", "pbh_get_stats", "pbh_walk_clock", "pbh_set_timing", "pbh_debug_tree",
           "pbh_debug_groups",
           "pbh_debug_wave_log", "pbh_debug_valu_probe", "pbh_debug_herm_first_steps",
           "pbh_debug_series_log",
           "pbh_last_error", "pbh_status_string")


class pbh_params(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("n_crit", C.c_int32), ("walk_tile", C.c_int32),
                ("lanes_per_particle", C.c_int32), ("key_bits", C.c_int32), ("prec", C.c_int32)]


class pbh_stats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in (
        "n", "n_clusters", "n_nodes", "n_leaves", "n_groups", "max_level", "n_pn", "n_pp_far",
        "n_pp_near", "nbr_total", "error_flags")] + [
        (name, C.c_double) for name in ("ms_build", "ms_walk", "ms_nbr")] + [
        (name, C.c_int64) for name in ("lane_slots_pn", "lane_slots_far", "lane_slots_near")]


class pbh_core_info(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("rho_core", C.c_double), ("r_core", C.c_double),
                ("n_core", C.c_int64), ("r_half", C.c_double), ("r_min", C.c_double),
                ("dt_min", C.c_double)]


class PbhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pbh status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libpbh.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- loads the HIP runtime the library will bind to
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2110_11658_amd.build.build()")
    L = C.CDLL(path)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    st = C.c_int
    sig = {
        "pbh_create": (st, [C.c_int, vp, vp]),
        "pbh_destroy": (None, [vp]),
        "pbh_set_params": (st, [vp, vp]),
        "pbh_get_params": (st, [vp, vp]),
        "pbh_build": (st, [vp, i64, vp, vp, vp]),
        "pbh_force": (st, [vp, vp, vp, d, d, d, d, vp, vp, vp, vp, i64, vp, vp]),
        "pbh_build_batched": (st, [vp, i32, vp, vp, vp, vp]),
        "pbh_force_batched": (st, [vp, vp, vp, vp, vp, d, d, vp, vp, vp, vp, i64, vp, vp]),
        "pbh_force_buffered": (st, [vp, vp, vp, d, d, d, d, d, vp, vp, vp, vp, i64, vp, vp]),
        "pbh_force_batched_buffered": (st, [vp, vp, vp, vp, vp, vp, d, d, vp, vp, vp, vp, i64, vp,
                                            vp]),
        "pbh_irregular": (st, [vp, i64, vp, vp, vp, d, d, d, vp, vp, i64, i64, vp, vp, vp, vp,
                               i32, vp]),
        "pbh_irregular_batched": (st, [vp, vp, vp, vp, vp, vp, d, vp, vp, i64, i64, vp, vp, vp,
                                       vp, i32, vp]),
        "pbh_irregular_noalloc": (st, [vp, i64, vp, vp, vp, d, d, d, vp, vp, i64, i64, vp, vp, vp,
                                       vp, i32, vp]),
        "pbh_core": (st, [vp, vp, vp, i64, vp, d, vp, vp, vp]),
        "pbh_hermite": (st, [vp, i64, vp, vp, vp, vp, d, d, d, vp, vp, i64, d, d, vp, vp]),
        "pbh_p3t": (st, [vp, i64, vp, vp, vp, d, d, d, d, d, d, d, i32, vp, vp, vp]),
        "pbh_kdk_graph": (st, [vp, i64, vp, vp, vp, d, i32, d, d, d, d, vp, vp]),
        "pbh_kdk_eager": (st, [vp, i64, vp, vp, vp, d, i32, d, d, d, d, vp, vp]),
        "pbh_get_stats": (st, [vp, vp]),
        "pbh_walk_clock": (st, [vp, vp]),
        "pbh_set_timing": (st, [vp, i32]),
        "pbh_debug_tree": (st, [vp, vp, vp, i64, vp, vp, vp]),
        "pbh_debug_groups": (st, [vp, i64, vp, vp, vp, vp]),
        "pbh_debug_wave_log": (st, [vp, vp, vp, i64, vp, vp]),
        "pbh_debug_valu_probe": (st, [vp, i64, i32, vp, vp]),
        "pbh_debug_series_log": (st, [vp, i64, vp, vp, vp]),
        "pbh_debug_herm_first_steps": (st, [vp, i64, vp, vp]),
        "pbh_last_error": (C.c_char_p, [vp]),
        "pbh_status_string": (C.c_char_p, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(ctx, status: int):
    if status != PBH_OK:
        L = load()
        msg = L.pbh_last_error(ctx).decode() if ctx else L.pbh_status_string(status).decode()
        raise PbhError(status, msg)
