"""Batched mode (one persistent launch over many jobs) and serving mode
(continuous batching of streamed frames): thin wrappers over the xeng_plan_*
and xeng_server_* C ABI. Tensors are only marshalled; the library does the
work. Objects keep references to every tensor they hand to the library."""
from __future__ import annotations

import ctypes

from ._lib import XengError, XengJob, check, lib


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _cstr(path):
    return None if path is None else str(path).encode()


class Plan:
    """Many correlation jobs run by one persistent launch.

    jobs: list of (x uint8[F][T][N], vis int32[F][N(N+1)/2][2]) or
    (x, vis, t_prev, accumulate) tuples, all on the same GPU.
    workspace: False makes no device allocation at all; the plan then runs
    only through run_static (the library's static device array).
    """

    def __init__(self, jobs, tune_cache=None, workspace=True):
        import torch
        self._keep = []
        arr = (XengJob * len(jobs))()
        for k, job in enumerate(jobs):
            x, vis = job[0], job[1]
            t_prev = job[2] if len(job) > 2 else 0
            acc = job[3] if len(job) > 3 else False
            if x.dtype != torch.uint8 or vis.dtype != torch.int32 or not (x.is_cuda and vis.is_cuda):
                raise TypeError("job %d: need GPU uint8 input and int32 output" % k)
            f, t, n = x.shape
            arr[k] = XengJob(x.data_ptr(), vis.data_ptr(), n, f, t, int(t_prev), int(bool(acc)))
            self._keep += [x, vis]
        self._jobs = arr
        h = ctypes.c_void_p()
        check(lib().xeng_plan_create(ctypes.byref(h), arr, len(jobs), _cstr(tune_cache)))
        self._h = h
        self.workspace = None
        if workspace:
            nbytes = int(lib().xeng_plan_workspace_bytes(h))
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=jobs[0][0].device)
            check(lib().xeng_plan_upload(h, self._ws(), _stream()))

    def _ws(self):
        if self.workspace is None:
            raise XengError(-1, "plan made without a workspace: use run_static()")
        return ctypes.c_void_p(self.workspace.data_ptr())

    @property
    def items(self) -> int:
        return int(lib().xeng_plan_items(self._h))

    @property
    def split(self) -> int:
        return int(lib().xeng_plan_split(self._h))

    def run(self, stream=None):
        check(lib().xeng_plan_run(self._h, self._ws(), _stream(stream)))

    def run_static(self, stream=None):
        """Run through the library's static device array (no workspace, no
        allocation); calls that overlap on one GPU race."""
        check(lib().xeng_plan_run_static(self._h, _stream(stream)))

    def set_frame(self, inputs=None, accumulate=True, stream=None):
        """Rebind every job to a new frame of inputs (same shapes)."""
        ptrs = None
        if inputs is not None:
            if len(inputs) != len(self._jobs):
                raise ValueError("one input per job")
            ptrs = (ctypes.c_void_p * len(inputs))(*[x.data_ptr() for x in inputs])
            self._keep += list(inputs)
        ws = None if self.workspace is None else self._ws()
        check(lib().xeng_plan_set_frame(self._h, ptrs, int(bool(accumulate)), ws,
                                        _stream(stream)))

    def capture_graph(self):
        check(lib().xeng_plan_graph_capture(self._h, self._ws()))

    def replay(self, stream=None):
        check(lib().xeng_plan_graph_launch(self._h, _stream(stream)))

    def autotune(self, reps: int = 3, tune_cache=None, stream=None) -> float:
        ms = ctypes.c_float(0.0)
        check(lib().xeng_plan_autotune(self._h, self._ws(), _stream(stream), int(reps),
                                       _cstr(tune_cache), ctypes.byref(ms)))
        return float(ms.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().xeng_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over device-resident accumulators."""

    def __init__(self, hbm_budget: int, max_inflight: int = 2, ws_bytes: int = 32 << 20,
                 device="cuda", stream=None):
        import torch
        self.workspace = torch.empty(int(ws_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(lib().xeng_server_create(ctypes.byref(h), int(hbm_budget), int(max_inflight),
                                       ctypes.c_void_p(self.workspace.data_ptr()), int(ws_bytes),
                                       _stream(stream)))
        self._h = h
        self._frames = {}
        self._acc = {}

    def open_job(self, n: int, f: int, vis) -> int:
        jid = ctypes.c_int64()
        check(lib().xeng_job_open(self._h, int(n), int(f), ctypes.c_void_p(vis.data_ptr()),
                                  ctypes.byref(jid)))
        self._acc[jid.value] = vis
        return jid.value

    def submit(self, job_id: int, frame) -> int:
        """frame: uint8[F][T][N] on the GPU, kept alive until its ticket is done."""
        tk = ctypes.c_uint64()
        t = frame.shape[1]
        check(lib().xeng_submit(self._h, int(job_id), ctypes.c_void_p(frame.data_ptr()), int(t),
                                ctypes.byref(tk)))
        self._frames[tk.value] = frame
        return tk.value

    def step(self) -> int:
        n = ctypes.c_int(0)
        check(lib().xeng_server_step(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, ticket: int):
        done = ctypes.c_int(0)
        lat = ctypes.c_double(-1.0)
        check(lib().xeng_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done),
                              ctypes.byref(lat)))
        if done.value:
            self._frames.pop(ticket, None)
        return bool(done.value), float(lat.value)

    def drain(self):
        check(lib().xeng_server_drain(self._h))

    def close_job(self, job_id: int):
        check(lib().xeng_job_close(self._h, int(job_id)))
        self._acc.pop(job_id, None)

    def stats(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        d = ctypes.c_size_t()
        check(lib().xeng_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                      ctypes.byref(d)))
        return {"open_jobs": a.value, "pending_frames": b.value, "inflight_steps": c.value,
                "bytes_in_use": d.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().xeng_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Plan", "Server", "XengError"]
