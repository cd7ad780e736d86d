"""Request loop for the serving mode: replay a stream of correlation frames
arriving at given times through the library's continuous-batching server,
and report throughput and frame latency.

Each (N, F) shape of the stream is one job whose int32 accumulator stays in
HBM for the whole run; frames are taken from a small pool of device-resident
buffers per shape (their contents only matter to correctness tests, not to
timing). The loop submits every frame whose arrival time has passed, lets the
server launch what it can (xeng_server_step), and polls for completions; the
library timestamps completions on the device, so polling speed does not bias
the latencies.
"""
from __future__ import annotations

import time

import numpy as np

from . import metrics
from .batch import Server


def run_stream(arrival_s, ns, fs, t: int, frames_for, hbm_budget: int, max_inflight: int = 2,
               ws_bytes: int = 64 << 20, device="cuda", time_limit_s: float = 60.0):
    """Serve frames k = 0.. arriving at arrival_s[k] (seconds from start) with
    shape (fs[k], t, ns[k]). frames_for(n, f) returns a list of device buffers
    uint8[f][t][n] to draw frames from. Returns a dict of statistics."""
    import torch

    shapes = sorted({(int(n), int(f)) for n, f in zip(ns, fs)})
    srv = Server(hbm_budget=hbm_budget, max_inflight=max_inflight, ws_bytes=ws_bytes,
                 device=device)
    acc = {}
    jobs = {}
    for n, f in shapes:
        acc[(n, f)] = torch.zeros((f, metrics.vis_entries(n), 2), dtype=torch.int32, device=device)
        jobs[(n, f)] = srv.open_job(n, f, acc[(n, f)])
    pools = {s: frames_for(*s) for s in shapes}
    torch.cuda.synchronize()
    total = len(arrival_s)
    tickets = [None] * total
    lat = np.full(total, np.nan)
    pending = []
    use = {s: 0 for s in shapes}
    i = 0
    done = 0
    peak_bytes = 0
    peak_pending = 0
    t0 = time.perf_counter()
    while done < total:
        now = time.perf_counter() - t0
        if now > time_limit_s:
            break
        while i < total and arrival_s[i] <= now:
            s = (int(ns[i]), int(fs[i]))
            buf = pools[s][use[s] % len(pools[s])]
            use[s] += 1
            tickets[i] = srv.submit(jobs[s], buf)
            pending.append(i)
            i += 1
        srv.step()
        st = srv.stats()
        peak_bytes = max(peak_bytes, st["bytes_in_use"])
        peak_pending = max(peak_pending, st["pending_frames"])
        still = []
        for k in pending:
            ok, l_us = srv.poll(tickets[k])
            if ok:
                lat[k] = l_us
                done += 1
            else:
                still.append(k)
        pending = still
        if i < total and not pending:
            # nothing in flight: sleep until the next arrival
            wait = arrival_s[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    wall = time.perf_counter() - t0
    srv.drain()
    ops = sum(metrics.effective_ops(int(n), int(f), t) for n, f in zip(ns[:done], fs[:done]))
    served = lat[~np.isnan(lat)]
    stats = {
        "frames": int(total),
        "completed": int(done),
        "wall_s": wall,
        "offered_rate_hz": float(total / max(arrival_s[-1], 1e-9)) if total > 1 else None,
        "throughput_tops": ops / wall / 1e12,
        "frames_per_s": done / wall,
        "p50_latency_ms": float(np.percentile(served, 50) / 1e3) if served.size else None,
        "p99_latency_ms": float(np.percentile(served, 99) / 1e3) if served.size else None,
        "max_latency_ms": float(served.max() / 1e3) if served.size else None,
        "hbm_budget_bytes": int(hbm_budget),
        "peak_bytes_in_use": int(peak_bytes),
        "peak_pending_frames": int(peak_pending),
    }
    srv.close()
    return stats, acc
