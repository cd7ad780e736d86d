"""ctypes loader for libxengine.so and the C ABI's signatures.

There is no fallback: if the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxengine.so")

XENG_OK = 0
STATUS_NAMES = {0: "XENG_OK", -1: "XENG_EINVAL", -2: "XENG_ERANGE", -3: "XENG_ENOMEM",
                -4: "XENG_EDEVICE", -5: "XENG_EBUSY", -6: "XENG_ENOTFOUND"}


class XengError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status
        self.message = message


_lib = None

c_i64 = ctypes.c_int64
c_int = ctypes.c_int
c_vp = ctypes.c_void_p
c_cp = ctypes.c_char_p
c_size = ctypes.c_size_t
c_u64 = ctypes.c_uint64
c_f32p = ctypes.POINTER(ctypes.c_float)
c_intp = ctypes.POINTER(ctypes.c_int)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_dblp = ctypes.POINTER(ctypes.c_double)
c_sizep = ctypes.POINTER(ctypes.c_size_t)


class XengJob(ctypes.Structure):
    """Mirror of struct xeng_job."""
    _fields_ = [("d_in", c_vp), ("d_vis", c_vp), ("n", c_int), ("f", c_int), ("t", c_int),
                ("t_prev", c_i64), ("accumulate", c_int)]

# name -> (restype, argtypes); one line per symbol declared in include/xengine.h
SIGNATURES = {
    "xeng_last_error": (c_cp, []),
    "xeng_version": (c_cp, []),
    "xeng_vis_entries": (c_i64, [c_int]),
    "xeng_tri_index": (c_i64, [c_int, c_int, c_int]),
    "xeng_tile_count": (c_i64, [c_int, c_int]),
    "xeng_correlate": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_i64, c_int, c_vp]),
    "xeng_variant_count": (c_int, []),
    "xeng_variant_name": (c_cp, [c_int]),
    "xeng_correlate_variant": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_i64, c_int, c_int,
                                       c_int, c_vp]),
    "xeng_choose_variant": (c_int, [c_int, c_int, c_int, c_int, c_intp, c_intp]),
    "xeng_correlate_strided": (c_int, [c_vp, c_i64, c_i64, c_vp, c_int, c_int, c_int, c_i64, c_int,
                                       c_vp]),
    "xeng_correlate_gated": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_int, c_int, c_vp, c_vp,
                                     c_int, c_vp]),
    "xeng_correlate_delayed": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_vp, c_int, c_i64, c_int,
                                       c_vp]),
    "xeng_delayed_workspace_bytes": (c_size, [c_int, c_int, c_int]),
    "xeng_correlate_delayed_ws": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_vp, c_int, c_i64,
                                          c_int, c_vp, c_size, c_vp]),
    "xeng_autotune": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_int, c_cp, c_intp, c_intp, c_f32p,
                              c_vp]),
    "xeng_tune_load": (c_int, [c_cp, c_intp]),
    "xeng_tune_clear": (None, []),
    "xeng_plan_create": (c_int, [ctypes.POINTER(c_vp), ctypes.POINTER(XengJob), c_int, c_cp]),
    "xeng_plan_workspace_bytes": (c_size, [c_vp]),
    "xeng_plan_items": (c_i64, [c_vp]),
    "xeng_plan_split": (c_int, [c_vp]),
    "xeng_plan_upload": (c_int, [c_vp, c_vp, c_vp]),
    "xeng_plan_set_frame": (c_int, [c_vp, ctypes.POINTER(c_vp), c_int, c_vp, c_vp]),
    "xeng_plan_run": (c_int, [c_vp, c_vp, c_vp]),
    "xeng_plan_run_static": (c_int, [c_vp, c_vp]),
    "xeng_plan_graph_capture": (c_int, [c_vp, c_vp]),
    "xeng_plan_graph_launch": (c_int, [c_vp, c_vp]),
    "xeng_plan_autotune": (c_int, [c_vp, c_vp, c_vp, c_int, c_cp, c_f32p]),
    "xeng_plan_destroy": (None, [c_vp]),
    "xeng_server_create": (c_int, [ctypes.POINTER(c_vp), c_size, c_int, c_vp, c_size, c_vp]),
    "xeng_job_open": (c_int, [c_vp, c_int, c_int, c_vp, c_i64p]),
    "xeng_submit": (c_int, [c_vp, c_i64, c_vp, c_int, c_u64p]),
    "xeng_server_step": (c_int, [c_vp, c_intp]),
    "xeng_poll": (c_int, [c_vp, c_u64, c_intp, c_dblp]),
    "xeng_server_drain": (c_int, [c_vp]),
    "xeng_job_close": (c_int, [c_vp, c_i64]),
    "xeng_server_stats": (c_int, [c_vp, c_i64p, c_i64p, c_i64p, c_sizep]),
    "xeng_server_destroy": (None, [c_vp]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libxengine.so is not built (run __graft_entry__.build() or "
                              "python -m paper_1503_06203_amd.build); there is no CPU fallback")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != XENG_OK:
        raise XengError(status, lib().xeng_last_error().decode())
