"""MI355X (gfx950) 4-bit X-engine: cross-correlation of Excess-8 complex samples.

Thin Python binding over the C ABI in include/xengine.h. Every step of the
correlation runs in the library's HIP kernels; this module only checks tensor
types and passes device pointers and the current HIP stream. PyTorch provides
device memory and streams.

    x   = torch.uint8  [F][T][N] on the GPU  (high nibble Re+8, low nibble Im+8)
    vis = torch.int32  [F][N(N+1)/2][2]      (re, im), row-major upper triangle
    correlate(x, vis)                         # V_ij = sum_t x_i(t) conj(x_j(t))
"""
from __future__ import annotations

from . import metrics
from ._lib import XengError, check, lib

__all__ = ["correlate", "correlate_variant", "correlate_gated", "correlate_delayed",
           "choose_variant", "autotune", "tune_load", "tune_clear", "new_vis", "vis_entries",
           "tri_index", "tile_count", "variants", "XengError", "metrics", "MAX_SAMPLES", "Plan",
           "Server"]


def __getattr__(name):
    # batched / serving wrappers, imported on first use
    if name in ("Plan", "Server"):
        from . import batch
        return getattr(batch, name)
    raise AttributeError(name)

MAX_SAMPLES = metrics.MAX_SAMPLES


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes_void(stream.cuda_stream)


def ctypes_void(v):
    import ctypes
    return ctypes.c_void_p(int(v))


def _check_tensors(x, vis):
    import torch
    if x.dtype != torch.uint8 or x.dim() != 3:
        raise TypeError("x must be a uint8 tensor [F][T][N]")
    if vis.dtype != torch.int32:
        raise TypeError("vis must be an int32 tensor [F][N(N+1)/2][2]")
    if not (x.is_cuda and vis.is_cuda):
        raise TypeError("x and vis must be GPU tensors (the library has no CPU path)")
    if not vis.is_contiguous():
        raise TypeError("vis must be contiguous")
    if x.numel() and x.stride(2) != 1:
        raise TypeError("x: the elements of one sample must be contiguous (stride 1)")
    f, t, n = x.shape
    if vis.numel() != 2 * f * vis_entries(n):
        raise ValueError("vis must hold F*N(N+1)/2 (re, im) pairs")
    return f, t, n


def _dense(x):
    f, t, n = x.shape
    return x.is_contiguous() or (x.stride(1) == n and x.stride(0) == t * n) or x.numel() == 0


def correlate(x, vis, t_prev: int = 0, accumulate: bool = False, stream=None):
    """Correlate x into vis on the GPU (enqueued on ``stream``, default current).

    x may be any [F][T][N] view whose elements are contiguous, e.g. a time-major
    stream [T][F][N] seen as ``stream.permute(1, 0, 2)``: it is read in place."""
    f, t, n = _check_tensors(x, vis)
    if _dense(x):
        check(lib().xeng_correlate(x.data_ptr() if t else None, vis.data_ptr(), n, f, t,
                                   int(t_prev), int(bool(accumulate)), _stream_ptr(stream)))
    else:
        check(lib().xeng_correlate_strided(x.data_ptr(), int(x.stride(1)), int(x.stride(0)),
                                           vis.data_ptr(), n, f, t, int(t_prev),
                                           int(bool(accumulate)), _stream_ptr(stream)))
    return vis


def correlate_variant(x, vis, variant: int, split_t: int = 1, t_prev: int = 0,
                      accumulate: bool = False, stream=None):
    """Same as correlate() with an explicit kernel variant and time split (dense x)."""
    f, t, n = _check_tensors(x, vis)
    if not _dense(x):
        raise TypeError("correlate_variant needs a dense [F][T][N] input")
    check(lib().xeng_correlate_variant(x.data_ptr() if t else None, vis.data_ptr(), n, f, t,
                                       int(t_prev), int(bool(accumulate)), int(variant),
                                       int(split_t), _stream_ptr(stream)))
    return vis


def correlate_gated(x, vis, gate_of_block, block: int, t_prev=None, accumulate: bool = False,
                    stream=None):
    """Gated correlation: vis is int32 [G][F][N(N+1)/2][2]; block k of ``block``
    samples goes to gate gate_of_block[k] (0xFF leaves it out). t_prev: samples
    already held per gate (accumulating)."""
    import ctypes

    import numpy as np
    import torch
    if x.dtype != torch.uint8 or x.dim() != 3 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous GPU uint8 tensor [F][T][N]")
    if vis.dtype != torch.int32 or vis.dim() != 4 or not vis.is_cuda or not vis.is_contiguous():
        raise TypeError("vis must be a contiguous GPU int32 tensor [G][F][N(N+1)/2][2]")
    f, t, n = x.shape
    gates = vis.shape[0]
    if tuple(vis.shape[1:]) != (f, vis_entries(n), 2):
        raise ValueError("vis must be [G][F][N(N+1)/2][2]")
    g = np.ascontiguousarray(np.asarray(gate_of_block, dtype=np.uint8))
    if g.size < (t + block - 1) // block:
        raise ValueError("gate_of_block needs ceil(T / block) entries")
    tp = None
    if accumulate:
        tp = np.ascontiguousarray(np.asarray(t_prev if t_prev is not None else [0] * gates,
                                             dtype=np.int64))
    check(lib().xeng_correlate_gated(
        x.data_ptr() if t else None, vis.data_ptr(), int(gates), n, f, t, int(block),
        g.ctypes.data_as(ctypes.c_void_p), tp.ctypes.data_as(ctypes.c_void_p) if tp is not None else None,
        int(bool(accumulate)), _stream_ptr(stream)))
    return vis


def correlate_delayed(x, vis, delays, t_prev: int = 0, accumulate: bool = False, stream=None,
                      workspace=None):
    """Delay compensation: x is uint8 [F][T + D][N] with D = max(delays) halo
    samples first; element e's frame sample s is x[:, D + s - delays[e], e].
    vis int32 [F][N(N+1)/2][2] as for correlate(). Shapes the fused triangle
    kernels take (N <= 256, T % 64 == 0) need no workspace; others shift the
    samples into a workspace first (a uint8 GPU tensor; None allocates one
    pass's worth)."""
    import ctypes

    import numpy as np
    import torch
    if x.dtype != torch.uint8 or x.dim() != 3 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous GPU uint8 tensor [F][T + D][N]")
    d = np.ascontiguousarray(np.asarray(delays, dtype=np.int32))
    f, tt, n = x.shape
    if d.shape != (n,):
        raise ValueError("delays needs one entry per element")
    dmax = int(d.max()) if n else 0
    t = tt - dmax
    if vis.dtype != torch.int32 or not vis.is_cuda or not vis.is_contiguous() or \
            vis.numel() != 2 * f * vis_entries(n):
        raise TypeError("vis must be a contiguous GPU int32 tensor [F][N(N+1)/2][2]")
    need = int(lib().xeng_delayed_workspace_bytes(n, f, t))
    if need == 0 and workspace is None and n <= 256:
        check(lib().xeng_correlate_delayed(x.data_ptr(), vis.data_ptr(), n, f, t,
                                           d.ctypes.data_as(ctypes.c_void_p), dmax, int(t_prev),
                                           int(bool(accumulate)), _stream_ptr(stream)))
        return vis
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    if workspace is not None and (workspace.dtype != torch.uint8 or not workspace.is_cuda or
                                  not workspace.is_contiguous()):
        raise TypeError("workspace must be a contiguous GPU uint8 tensor")
    ws_ptr = workspace.data_ptr() if workspace is not None and workspace.numel() else None
    ws_len = workspace.numel() if workspace is not None else 0
    check(lib().xeng_correlate_delayed_ws(x.data_ptr(), vis.data_ptr(), n, f, t,
                                          d.ctypes.data_as(ctypes.c_void_p), dmax, int(t_prev),
                                          int(bool(accumulate)), ws_ptr, ws_len,
                                          _stream_ptr(stream)))
    return vis


def autotune(x, vis, reps: int = 3, tune_cache=None, stream=None):
    """Time every kernel variant (and time split) that can correlate x into
    vis, remember the fastest for this job class (device, N, F, log2 T) in the
    library and optionally append it to the file tune_cache. vis receives the
    correlation of x. Returns (variant id, split_t, milliseconds)."""
    import ctypes
    f, t, n = _check_tensors(x, vis)
    if not x.is_contiguous():
        raise TypeError("autotune needs a dense [F][T][N] input")
    v, sp, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    check(lib().xeng_autotune(x.data_ptr(), vis.data_ptr(), n, f, t, int(reps),
                              None if tune_cache is None else str(tune_cache).encode(),
                              ctypes.byref(v), ctypes.byref(sp), ctypes.byref(ms),
                              _stream_ptr(stream)))
    return v.value, sp.value, ms.value


def tune_load(tune_cache) -> int:
    """Load tuned choices from a file written by autotune(); returns how many
    apply to this device."""
    import ctypes
    k = ctypes.c_int()
    check(lib().xeng_tune_load(str(tune_cache).encode(), ctypes.byref(k)))
    return k.value


def tune_clear() -> None:
    lib().xeng_tune_clear()


def choose_variant(n: int, f: int, t: int, aligned: bool = True):
    """(variant id, time split, variant name) that correlate() uses for a job
    of this shape; aligned = the input pointer is 4-byte aligned."""
    import ctypes
    v, sp = ctypes.c_int(), ctypes.c_int()
    check(lib().xeng_choose_variant(int(n), int(f), int(t), int(bool(aligned)), ctypes.byref(v),
                                    ctypes.byref(sp)))
    return v.value, sp.value, variants()[v.value]


def new_vis(n: int, f: int, device="cuda"):
    import torch
    return torch.zeros((f, vis_entries(n), 2), dtype=torch.int32, device=device)


def vis_entries(n: int) -> int:
    return int(lib().xeng_vis_entries(int(n)))


def tri_index(n: int, i: int, j: int) -> int:
    return int(lib().xeng_tri_index(int(n), int(i), int(j)))


def tile_count(n: int, tile: int) -> int:
    return int(lib().xeng_tile_count(int(n), int(tile)))


def variants():
    L = lib()
    return [L.xeng_variant_name(k).decode() for k in range(L.xeng_variant_count())]
