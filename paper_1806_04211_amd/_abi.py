"""ctypes declarations of the C ABI in include/gfech.h (argument marshalling only)."""
from __future__ import annotations

import ctypes

c_i64 = ctypes.c_int64
c_u32 = ctypes.c_uint32
c_i32 = ctypes.c_int32
u8p = ctypes.POINTER(ctypes.c_uint8)
i64p = ctypes.POINTER(ctypes.c_int64)
vp = ctypes.c_void_p

GFECH_OK = 0
GFECH_E_STATE = 8
# what a call computes (gfech_opts.variant)
WANT_RREF_T, WANT_RREF, WANT_RANK = 0, 1, 2
STATUS_NAMES = {0: "GFECH_OK", 1: "GFECH_E_ARG", 2: "GFECH_E_FIELD", 3: "GFECH_E_RANGE", 4: "GFECH_E_NOMEM",
                5: "GFECH_E_TOO_BIG", 6: "GFECH_E_DEVICE", 7: "GFECH_E_CANCELLED", 8: "GFECH_E_STATE"}


class Opts(ctypes.Structure):
    _fields_ = [("block_rows", c_i64), ("block_cols", c_i64), ("skip_range_check", c_i32),
                ("profile", c_i32), ("variant", c_i32), ("timeout_ms", c_i32), ("reserved", c_i32 * 4)]


class Problem(ctypes.Structure):
    _fields_ = [("A", vp), ("m", c_i64), ("n", c_i64), ("lda", c_i64), ("p", c_u32), ("reserved", c_u32)]


class View(ctypes.Structure):
    _fields_ = [("R", vp), ("ldr", c_i64), ("M", vp), ("ldm", c_i64), ("K", vp), ("ldk", c_i64),
                ("gamma", vp), ("gamma_bar", vp), ("rho", vp), ("rho_bar", vp)]


class Stats(ctypes.Structure):
    _fields_ = [("mac_cleardown", ctypes.c_double), ("mac_ech", ctypes.c_double),
                ("mac_updaterow", ctypes.c_double), ("mac_trafo", ctypes.c_double),
                ("mac_clearup", ctypes.c_double), ("gather_bytes", ctypes.c_double),
                ("layers", c_i64), ("echs", c_i64), ("gemms", c_i64), ("launches", c_i64), ("syncs", c_i64),
                ("block_rows", c_i64), ("block_cols", c_i64),
                ("ms_mad", ctypes.c_double), ("ms_ech", ctypes.c_double), ("ms_small", ctypes.c_double),
                ("launches_mad", c_i64), ("launches_ech", c_i64), ("launches_small", c_i64),
                ("mad_bytes", ctypes.c_double), ("mac_mad_timed", ctypes.c_double), ("variant", c_i64),
                ("tail_checks", c_i64), ("ech_reruns", c_i64)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_i64), ("max_active", c_i32), ("size_classes", c_i32), ("reserved", c_i32 * 4)]


class Blocking(ctypes.Structure):
    _fields_ = [("max_dim", c_i64), ("block_rows", c_i64), ("block_cols", c_i64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("peak_bytes_in_flight", c_i64), ("peak_active", c_i64), ("admitted", c_i64), ("finished", c_i64)]


class MadDesc(ctypes.Structure):
    _fields_ = [("M", c_i64), ("N", c_i64), ("K", c_i64), ("p", c_u32), ("reserved", c_u32),
                ("A", vp), ("lda", c_i64), ("B", vp), ("ldb", c_i64), ("brow", vp),
                ("C", vp), ("ldc", c_i64), ("crow", vp), ("D", vp), ("ldd", c_i64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "gfech_echelonise_u8": (ctypes.c_int, [vp, c_i64, c_i64, c_i64, c_u32, vp, ctypes.POINTER(vp)]),
    "gfech_echelonise_u8_dev": (ctypes.c_int, [vp, c_i64, c_i64, c_i64, c_u32, vp, vp, ctypes.POINTER(vp)]),
    "gfech_set_blocking": (ctypes.c_int, [vp, c_i64]),
    "gfech_echelonise_gf2": (ctypes.c_int, [vp, c_i64, c_i64, c_i64, vp, ctypes.POINTER(vp)]),
    "gfech_echelonise_gf2_dev": (ctypes.c_int, [vp, c_i64, c_i64, c_i64, vp, vp, ctypes.POINTER(vp)]),
    "gfech_echelonise_batch": (ctypes.c_int, [c_i64, vp, c_i32, vp, vp, ctypes.POINTER(vp), vp]),
    "gfech_rank": (c_i64, [vp]),
    "gfech_shape": (ctypes.c_int, [vp, i64p, i64p, ctypes.POINTER(c_u32)]),
    "gfech_pivots": (ctypes.c_int, [vp, vp, vp]),
    "gfech_nonpivots": (ctypes.c_int, [vp, vp, vp]),
    "gfech_get_R": (ctypes.c_int, [vp, vp, c_i64]),
    "gfech_get_M": (ctypes.c_int, [vp, vp, c_i64]),
    "gfech_get_K": (ctypes.c_int, [vp, vp, c_i64]),
    "gfech_expand_rref": (ctypes.c_int, [vp, vp, c_i64]),
    "gfech_expand_transform": (ctypes.c_int, [vp, vp, c_i64]),
    "gfech_expand_rref_dev": (ctypes.c_int, [vp, vp, c_i64, vp]),
    "gfech_expand_transform_dev": (ctypes.c_int, [vp, vp, c_i64, vp]),
    "gfech_device_view": (ctypes.c_int, [vp, ctypes.POINTER(View)]),
    "gfech_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(Stats)]),
    "gfech_result_free": (None, [vp]),
    "gfech_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gfech_last_error": (ctypes.c_char_p, []),
    "gfech_backend_name": (ctypes.c_char_p, []),
    "gfech_mad_dev": (ctypes.c_int, [c_i64, c_i64, c_i64, c_u32, vp, c_i64, vp, c_i64, vp, vp, c_i64, vp, vp,
                                     c_i64, vp]),
    "gfech_mad_gf2_dev": (ctypes.c_int, [c_i64, c_i64, c_i64, vp, c_i64, vp, c_i64, vp, c_i64, vp, c_i64, vp]),
    "gfech_mad_batch_dev": (ctypes.c_int, [c_i64, vp, vp]),
    "gfech_mad_batch_dev_timed": (ctypes.c_int, [c_i64, vp, vp, ctypes.POINTER(ctypes.c_double)]),
    "gfech_ech_dev": (ctypes.c_int, [vp, c_i64, c_i64, c_i64, c_u32, vp, vp, vp, vp, vp, c_i64, vp, c_i64, vp,
                                     c_i64, i64p, vp]),
    "gfech_ech_dev_noalloc": (ctypes.c_int, [vp, c_i64, c_i64, c_i64, c_u32, vp, vp, vp, vp, vp, c_i64, vp, c_i64,
                                             vp, c_i64, vp, vp]),
    "gfech_server_create": (ctypes.c_int, [vp, ctypes.POINTER(vp)]),
    "gfech_server_submit": (ctypes.c_int, [vp, vp, c_i32, ctypes.POINTER(ctypes.c_uint64)]),
    "gfech_server_poll": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.POINTER(vp)]),
    "gfech_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
    "gfech_server_cancel": (ctypes.c_int, [vp, ctypes.c_uint64]),
    "gfech_server_wait": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.POINTER(vp)]),
    "gfech_server_destroy": (None, [vp]),
}


def declare(lib):
    """Attach the argument / result types to a loaded library; returns it."""
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
