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
