"""CPU oracle for the 4-bit X-engine cross-correlation (test infrastructure).

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark import this module. The GPU library neither imports nor links it,
and the two share no code.

The arithmetic lives in ``xcorr_oracle.c`` (plain loops, int64 sums). This
module builds that file with gcc, loads it with ctypes and adds numpy
wrappers. What it computes follows the paper:

* Sec. III, Excess-8 encoding: one byte per complex sample, each 4-bit field
  holds value + 8; the real part is the high nibble (the reading taken here).
* Sec. II-A, Eq. 1: V_ij = sum_t x_i(t) * conj(x_j(t)), kept for i <= j
  (Hermitian matrix, Eq. 2), in the row-major packed upper triangle.
* Sec. III, Eq. 3: the unsigned-product-plus-offset route, a second route to
  the same numbers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xcorr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None

INT32_MIN = -(2**31)
INT32_MAX = 2**31 - 1


def build(force: bool = True) -> str:
    """Compile xcorr_oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-Wall",
               "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.xcorr_oracle_correlate.argtypes = [u8p, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]
    lib.xcorr_oracle_full_matrix.argtypes = [u8p, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.xcorr_oracle_entries.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p,
                                         ctypes.c_int64, i64p]
    lib.xcorr_oracle_offset_route.argtypes = [u8p, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    for name in ("xcorr_oracle_correlate", "xcorr_oracle_full_matrix", "xcorr_oracle_entries",
                 "xcorr_oracle_offset_route", "xcorr_oracle_threads"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _u8(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i64(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _as_input(packed) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(packed), dtype=np.uint8)
    if a.ndim != 3:
        raise ValueError("packed input must be uint8[F][T][N]")
    return a


def vis_entries(n: int) -> int:
    """Entries of the packed upper triangle, n(n+1)/2 (Eq. 2)."""
    return n * (n + 1) // 2


def correlate(packed, prev: np.ndarray | None = None) -> np.ndarray:
    """Upper-triangle visibilities int64[F][n(n+1)/2][2] of uint8[F][T][N] input.

    With ``prev`` the new sums are added to it (Sec. III-A, results added to
    those already held).
    """
    x = _as_input(packed)
    f, t, n = x.shape
    out = np.zeros((f, vis_entries(n), 2), dtype=np.int64)
    acc = 0
    if prev is not None:
        out[...] = np.asarray(prev, dtype=np.int64).reshape(out.shape)
        acc = 1
    rc = _load().xcorr_oracle_correlate(_u8(x), _i64(out), n, f, t, acc)
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def full_matrix(packed) -> np.ndarray:
    """Every (i, j), lower triangle included: int64[F][N][N][2]."""
    x = _as_input(packed)
    f, t, n = x.shape
    out = np.zeros((f, n, n, 2), dtype=np.int64)
    rc = _load().xcorr_oracle_full_matrix(_u8(x), _i64(out), n, f, t)
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def entries(packed, fij) -> np.ndarray:
    """Selected entries (channel, i, j), i <= j, as int64[m][2]."""
    x = _as_input(packed)
    f, t, n = x.shape
    q = np.ascontiguousarray(np.asarray(fij, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((q.shape[0], 2), dtype=np.int64)
    rc = _load().xcorr_oracle_entries(_u8(x), n, f, t, _i64(q), q.shape[0], _i64(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def offset_route(packed) -> np.ndarray:
    """The same visibilities through the paper's Eq. 3 offset route."""
    x = _as_input(packed)
    f, t, n = x.shape
    out = np.zeros((f, vis_entries(n), 2), dtype=np.int64)
    rc = _load().xcorr_oracle_offset_route(_u8(x), _i64(out), n, f, t)
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return out


def correlate_gated(packed, gate_of_block, block: int, gates: int) -> np.ndarray:
    """Gated correlation: int64 [G][F][N(N+1)/2][2], gate g summing Eq. 1 over
    the samples whose block (of ``block`` samples, block k = samples
    k*block .. k*block+block-1) is assigned to g; 0xFF leaves a block out.
    Written from that definition: each gate's samples are gathered and
    correlated with the plain oracle above."""
    x = _as_input(packed)
    f, t, n = x.shape
    g = np.asarray(gate_of_block, dtype=np.int64)
    out = np.zeros((gates, f, vis_entries(n), 2), dtype=np.int64)
    sample_gate = np.repeat(g, block)[:t] if t else np.zeros(0, dtype=np.int64)
    for gate in range(gates):
        idx = np.nonzero(sample_gate == gate)[0]
        if idx.size:
            out[gate] = correlate(np.ascontiguousarray(x[:, idx, :]))
    return out


def correlate_delayed(packed, delays) -> np.ndarray:
    """Delay compensation (Sec. IV, elements shifted by whole time steps before
    correlation): packed is [F][T + D][N] with D = max(delays);
    returns the correlation of the aligned streams y_e(s) = x_e(D + s - d_e),
    s < T, written from that definition (gather, then the plain oracle)."""
    x = _as_input(packed)
    f, tt, n = x.shape
    d = np.asarray(delays, dtype=np.int64)
    dmax = int(d.max()) if n else 0
    t = tt - dmax
    rows = dmax - d[None, :] + np.arange(t)[:, None]          # [T][N] input sample per (s, e)
    y = x[:, rows, np.arange(n)[None, :]]                      # [F][T][N]
    return correlate(np.ascontiguousarray(y))


def threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(_load().xcorr_oracle_threads())


def to_int32(vis64: np.ndarray) -> np.ndarray:
    """Range-check int64 sums into int32 (the output type of the GPU path)."""
    v = np.asarray(vis64)
    if v.size and (v.min() < INT32_MIN or v.max() > INT32_MAX):
        raise OverflowError("visibility sum outside int32")
    return v.astype(np.int32)


def tri_pairs(n: int) -> np.ndarray:
    """(i, j) for every packed index k, in the row-major upper-triangle order."""
    i, j = np.triu_indices(n)
    return np.stack([i, j], axis=1)
