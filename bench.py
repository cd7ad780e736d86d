#!/usr/bin/env python3
"""Benchmark of the 4-bit X-engine hot path on one MI355X.

A step is one full correlation of one frame of synthetic input that is already
resident in HBM. The headline workload is the full-CHIME large-N frame
(N=2048 elements, F=16 channels, T=65536 samples per frame, four frames
summed into device-resident accumulators in turn): one library call per step.
Prints ONE JSON line:

  value        effective correlation TOPS = 8 * N(N+1)/2 * F * T / step time
               (paper Eq. 2 operation count; redundant work is never counted)
  roofline     the dominant kernel against the int8 MFMA peak, timed with HIP
               events on the stream it is launched on; traffic = HBM bytes per
               launch from the FETCH_SIZE / WRITE_SIZE counters recorded in
               profiles/ for the current kernel source (null otherwise)
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
  pathfinder, tiny, small_n, time_major, gated, delayed, bf6, batched, served
               secondary measurements (other shapes and entry points)

--workload runs one workload alone (for profiling): tiny, pathfinder, large_n,
small_n, batched, served, or large_n_delayed (the large-N frame with
per-element delays: the shift kernel, then the correlation).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0      # MI355X dense int8 MFMA, TOP/s
PEAK_FP6_TFLOPS = 10100.0    # MI355X dense fp6/fp4 MFMA, TFLOP/s
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s


# kernel symbol of each library variant (the name rocprofv3 reports)
KERNEL_OF_VARIANT = {   # first matching prefix wins
    "tile128": "xcorr_tile128_kernel",
    "tri256_w8_bf6": "xcorr_tri_bf6_kernel",
    "tri256": "xcorr_tri_kernel",
    "rect128x256_tri256_w8_bf6": "xcorr_rect_bf6_kernel",
    "rect128x256": "xcorr_rect_kernel",
    "small64": "xcorr_small_kernel",
}


def dispatched_kernel(n: int, f: int, t: int):
    """(kernel symbol, variant name, time split) the library runs for this shape."""
    import paper_1503_06203_amd as xe
    _, split, name = xe.choose_variant(n, f, t)
    for prefix, kern in KERNEL_OF_VARIANT.items():
        if name.startswith(prefix):
            return kern, name, split
    return name, name, split


# the source file of each kernel; its digest also covers the headers it includes
KERNEL_SOURCE = {
    "xcorr_rect_kernel": "xcorr_rect.hip",
    "xcorr_tri_kernel": "xcorr_tri.hip",
    "xcorr_small_kernel": "xcorr_small.hip",
    "xcorr_tri_bf6_kernel": "xcorr_tri_bf6.hip",
    "xcorr_tile128_kernel": "xcorr_tile.hip",
    "xcorr_shift_kernel": "xcorr_shift.hip",
    "xcorr_rect_bf6_kernel": "xcorr_rect_bf6.hip",
}


def kernel_source_digest(kernel: str) -> str:
    """Digest of the sources a kernel is compiled from (its file and the
    package headers it includes, transitively): recorded HBM counters apply
    only while it is unchanged."""
    csrc = os.path.join(ROOT, "paper_1503_06203_amd", "csrc")
    todo, seen = [KERNEL_SOURCE.get(kernel, "")], []
    while todo:
        name = todo.pop()
        path = os.path.join(csrc, name)
        if name in seen or not os.path.isfile(path):
            continue
        seen.append(name)
        todo += re.findall(r'#include "([^"]+)"', open(path).read())
    h = hashlib.sha256()
    for name in sorted(seen):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, digest: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters, as recorded in profiles/, if taken on the current kernel source."""
    pat = re.compile(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+workload:\s*(\S+)\s+"
                     r"kernel_source:\s*([0-9a-f]+)")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            m = pat.search(line)
            if m and m.group(2) == workload and m.group(3) == digest:
                return float(m.group(1))
    return None


def time_steps(step, steps: int, warmup: int):
    """Time `steps` calls of step() after `warmup` untimed ones.

    Returns (wall seconds for all steps, per-launch kernel seconds from HIP
    events recorded on the current stream around each launch)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        step()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [s.elapsed_time(e) / 1e3 for s, e in zip(starts, ends)]
    return wall, per


def bench_workload(w, steps: int, warmup: int):
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics

    dev = "cuda:0"
    frames = [synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, s, common=w.common, device=dev)
              for s in w.seeds()]
    vis = xe.new_vis(w.n, w.f, device=dev)
    state = {"k": 0}

    def step():
        # one frame per step; frames after the first add to the resident sums
        k = state["k"]
        x = frames[k % len(frames)]
        first = (k % len(frames)) == 0
        xe.correlate(x, vis, t_prev=0 if first else (k % len(frames)) * w.t, accumulate=not first)
        state["k"] = k + 1

    torch.cuda.synchronize()
    wall, per = time_steps(step, steps, warmup)
    ops = metrics.effective_ops(w.n, w.f, w.t)
    step_s = wall / steps
    kern_s = sum(per) / len(per)
    del frames
    torch.cuda.empty_cache()
    return {
        "value": ops / step_s / 1e12,
        "ms_per_step": step_s * 1e3,
        "kernel_ms": kern_s * 1e3,
        "kernel_tops": ops / kern_s / 1e12,
        "ops_per_step": ops,
        "input_bytes": metrics.input_bytes(w.n, w.f, w.t),
    }


def bench_time_major(w, steps: int, warmup: int):
    """The same workload delivered as the paper's time-major packet stream
    [T][F][N] (Sec. III, Fig. 2), correlated in place through strides."""
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics

    dense = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seeds()[0], common=w.common,
                                     device="cuda:0")
    view = dense.permute(1, 0, 2).contiguous().permute(1, 0, 2)
    del dense
    vis = xe.new_vis(w.n, w.f, device="cuda:0")
    wall, per = time_steps(lambda: xe.correlate(view, vis), steps, warmup)
    ops = metrics.effective_ops(w.n, w.f, w.t)
    kern_s = sum(per) / len(per)
    del view
    torch.cuda.empty_cache()
    return {"layout": "[T][F][N] read in place (sample stride F*N, channel stride N)",
            "value": round(ops / (wall / steps) / 1e12, 3), "unit": "TOPS",
            "ms_per_step": round(wall / steps * 1e3, 5), "kernel_ms": round(kern_s * 1e3, 5)}


def bench_gated(w, steps: int, warmup: int):
    """Pulsar-style gating of the workload: two gate bins over blocks of 1024
    samples, on-pulse (gate 0) one block in four, off-pulse (gate 1) the rest."""
    import numpy as np
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics

    block = 1024
    x = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seeds()[0], common=w.common,
                                 device="cuda:0")
    nb = (w.t + block - 1) // block
    sched = np.array([0 if k % 4 == 0 else 1 for k in range(nb)], dtype=np.uint8)
    vis = torch.zeros((2, w.f, xe.vis_entries(w.n), 2), dtype=torch.int32, device="cuda:0")
    wall, _ = time_steps(lambda: xe.correlate_gated(x, vis, sched, block), steps, warmup)
    ops = metrics.effective_ops(w.n, w.f, w.t)
    del x, vis
    torch.cuda.empty_cache()
    runs = [0, 0]
    for k in range(nb):
        if k == 0 or sched[k] != sched[k - 1]:
            runs[int(sched[k])] += 1
    # all runs of one gate go to one launch (up to 32 runs per launch)
    launches = sum((r + 31) // 32 for r in runs)
    return {"workload": w.name, "n": w.n, "f": w.f, "t": w.t,
            "gates": 2, "block_samples": block, "schedule": "gate 0 one block in four, else gate 1",
            "runs_per_step": sum(runs), "launches_per_step": launches,
            "value": round(ops / (wall / steps) / 1e12, 3), "unit": "TOPS",
            "ms_per_step": round(wall / steps * 1e3, 5)}


def bench_delayed(w, steps: int, warmup: int, main_only: bool = False):
    """Delay compensation on the workload: per-element integer delays drawn
    uniformly from [0, 64] samples (the first element takes the largest), a
    64-sample halo in front of each channel. For comparison the same call with
    all delays equal (a shifted sample window, run on the dense kernel) and
    with delays 63 and 64 alternating (the smallest spread the window form
    stages), unless main_only. The effective rate counts the frame's samples
    only."""
    import numpy as np
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics

    dmax = 64
    x = synth.quantized_gaussian(w.f, w.t + dmax, w.n, w.sigma, w.seeds()[0], common=w.common,
                                 device="cuda:0")
    rng = np.random.default_rng(7)
    delays = rng.integers(0, dmax + 1, w.n).astype(np.int32)
    delays[0] = dmax
    vis = xe.new_vis(w.n, w.f)
    ops = metrics.effective_ops(w.n, w.f, w.t)
    need = int(xe.lib().xeng_delayed_workspace_bytes(w.n, w.f, w.t))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0") if need else None
    out = {"workload": w.name, "n": w.n, "f": w.f, "t": w.t, "max_delay": dmax,
           "delays": "uniform integers in [0, %d]" % dmax,
           "form": "shift into a %d-byte workspace, then correlate" % need if need
           else "fused into the triangle kernel's staging"}
    wall, per = time_steps(lambda: xe.correlate_delayed(x, vis, delays, workspace=ws), steps,
                           warmup)
    out.update({"value": round(ops / (wall / steps) / 1e12, 3), "unit": "TOPS",
                "ms_per_step": round(wall / steps * 1e3, 5)})
    if main_only:
        del x, vis, ws
        torch.cuda.empty_cache()
        return out
    same = np.full(w.n, dmax, dtype=np.int32)     # the same input, no relative shift
    wall0, _ = time_steps(lambda: xe.correlate_delayed(x, vis, same, workspace=ws), steps, warmup)
    out["equal_delays_value"] = round(ops / (wall0 / steps) / 1e12, 3)
    near = np.full(w.n, dmax, dtype=np.int32)
    near[1::2] = dmax - 1                         # spread 1
    wall1, _ = time_steps(lambda: xe.correlate_delayed(x, vis, near, workspace=ws), steps, warmup)
    out["spread1_value"] = round(ops / (wall1 / steps) / 1e12, 3)
    plain = xe.new_vis(w.n, w.f)
    wall2, _ = time_steps(lambda: xe.correlate(x[:, dmax:], plain), steps, warmup)
    out["no_delays_plain_value"] = round(ops / (wall2 / steps) / 1e12, 3)
    del x, vis, ws, plain
    torch.cuda.empty_cache()
    return out


def bench_bf6(w, steps: int, warmup: int, variant: int = 4):
    """The exact bf6 path (the triangle kernel, variant 4, or the kernel of
    squares and tiles, variant 7, on the f8f6f4 matrix cores) on the workload,
    reported apart from the int8 metric: its roofline is the fp6 peak. Also
    checks that its result equals the default path's bit for bit."""
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics

    x = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seeds()[0], common=w.common,
                                 device="cuda:0")
    vis = xe.new_vis(w.n, w.f)
    wall, per = time_steps(lambda: xe.correlate_variant(x, vis, variant, split_t=0), steps, warmup)
    ref = xe.correlate(x, xe.new_vis(w.n, w.f))
    torch.cuda.synchronize()
    same = bool(torch.equal(ref, vis))
    ops = metrics.effective_ops(w.n, w.f, w.t)
    kern_s = sum(per) / len(per)
    del x, vis, ref
    torch.cuda.empty_cache()
    achieved = ops / kern_s / 1e12
    return {"workload": w.name, "variant": xe.variants()[variant],
            "dtype": "bf6 (E3M2), fp32 accumulate",
            "value": round(ops / (wall / steps) / 1e12, 3), "unit": "TOPS",
            "ms_per_step": round(wall / steps * 1e3, 5), "kernel_ms": round(kern_s * 1e3, 5),
            "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                         "peak": PEAK_FP6_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / PEAK_FP6_TFLOPS, 4)},
            "identical_to_int8_path": same}


def cpu_baseline(w, budget_s: float = 15.0):
    """Time the CPU oracle on a bounded sample of the workload: one channel
    (all N elements) over a prefix of its samples, doubled from a short first
    run until one run takes at least a sixth of budget_s or covers the whole
    channel; then as many whole channels as fit half the budget. The last
    timed run is the reported sample (its own rate, nothing extrapolated)."""
    import numpy as np

    import oracle
    import synth
    from paper_1503_06203_amd import metrics

    oracle.build(force=False)
    drawn = {}

    def timed(k, t):
        if drawn.get("k", 0) < k:      # the workload's first k channels, drawn on the host
            drawn["x"] = synth.quantized_gaussian(k, w.t, w.n, w.sigma, w.seeds()[0],
                                                  common=w.common).numpy()
            drawn["k"] = k
        sample = np.ascontiguousarray(drawn["x"][:k, :t, :])
        t0 = time.perf_counter()
        oracle.correlate(sample)
        return time.perf_counter() - t0

    # the oracle's time per sample grows with the sample count (its working set
    # leaves the caches), so the prefix at most doubles per run
    k, t_use = 1, min(w.t, 1024)
    dt = timed(k, t_use)
    while dt < budget_s / 6 and t_use < w.t:
        t_use = min(w.t, 2 * t_use)
        dt = timed(k, t_use)
    if t_use == w.t and dt < budget_s / 3 and w.f > 1:
        k = int(max(1, min(w.f, 0.5 * budget_s / max(dt, 1e-3))))
        if k > 1:
            dt = timed(k, t_use)
    ops = metrics.effective_ops(w.n, k, t_use)
    return {"value": ops / dt / 1e12, "unit": "TOPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d of %d channels, N=%d, first %d of %d samples, first frame "
                      "(%.3g effective ops in %.2f s)" % (k, w.f, w.n, t_use, w.t, ops, dt)}


def mfma_roofline(w, r):
    """Roofline object for an MFMA-bound workload measured by bench_workload."""
    kern, vname, vsplit = dispatched_kernel(w.n, w.f, w.t)
    digest = kernel_source_digest(kern)
    return {
        "bound": "mfma",
        "achieved": round(r["kernel_tops"], 3),
        "peak": PEAK_INT8_TOPS,
        "unit": "TOP/s",
        "frac": round(r["kernel_tops"] / PEAK_INT8_TOPS, 4),
        "traffic": recorded_traffic(w.name, digest),
        "kernel": kern,
        "variant": vname,
        "time_split": vsplit,
        "kernel_ms": round(r["kernel_ms"], 5),
        "algorithmic_ops_per_launch": r["ops_per_step"],
        "input_gbs": round(r["input_bytes"] / (r["kernel_ms"] / 1e3) / 1e9, 1),
        "kernel_source": digest,
    }


def bench_small_n(w, steps: int, warmup: int):
    """A small array (N=64): bound by HBM rather than the matrix cores. The
    roofline is the algorithmic bytes (input read once, output written once)
    per launch over the launch time, against 8 TB/s."""
    from paper_1503_06203_amd import metrics

    r = bench_workload(w, steps, warmup)
    kern, vname, vsplit = dispatched_kernel(w.n, w.f, w.t)
    digest = kernel_source_digest(kern)
    alg = metrics.algorithmic_bytes(w.n, w.f, w.t, accumulate=False)
    gbs = alg / (r["kernel_ms"] / 1e3) / 1e9
    copy_gbs = copy_ceiling_gbs(w.f * w.t * w.n)
    return {"workload": w.name, "n": w.n, "f": w.f, "t": w.t,
            "value": round(r["value"], 3), "unit": "TOPS",
            "ms_per_step": round(r["ms_per_step"], 5),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                         "traffic": recorded_traffic(w.name, digest), "kernel": kern,
                         "variant": vname, "time_split": vsplit,
                         "kernel_ms": round(r["kernel_ms"], 5),
                         "algorithmic_bytes_per_launch": alg,
                         "mfma_frac": round(r["kernel_tops"] / PEAK_INT8_TOPS, 4),
                         "copy_ceiling_gbs": round(copy_gbs, 1),
                         "frac_of_copy": round(gbs / copy_gbs, 4)}}


def copy_ceiling_gbs(nbytes: int, reps: int = 10) -> float:
    """A measured stream ceiling on this device: bytes moved per second (read
    plus write) by a device-to-device copy of nbytes, best of reps."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    best = float("inf")
    for k in range(reps + 2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        b.synchronize()
        if k >= 2:
            best = min(best, a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (best / 1e3) / 1e9


def bench_autotune(w, r):
    """The autotuner on the workload's frame: the variant and split it keeps
    and its time against the default choice's launch time from the headline
    run. The choice is forgotten afterwards."""
    import torch

    import paper_1503_06203_amd as xe
    import synth

    x = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seeds()[0], common=w.common,
                                 device="cuda:0")
    vis = xe.new_vis(w.n, w.f, device="cuda:0")
    t0 = time.perf_counter()
    v, split, ms = xe.autotune(x, vis, reps=2)
    wall = time.perf_counter() - t0
    xe.tune_clear()
    del x, vis
    torch.cuda.empty_cache()
    return {"workload": w.name, "variant": xe.variants()[v], "split": split,
            "tuned_ms": round(ms, 5), "default_kernel_ms": round(r["kernel_ms"], 5),
            "search_s": round(wall, 2)}


def bench_latency(w, calls: int = 200):
    """Latency of one small correlation (the tiny workload): device time per
    launch from HIP events, and host time of one call followed by a wait."""
    import torch

    import paper_1503_06203_amd as xe
    import synth

    x = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seed, device="cuda:0")
    vis = xe.new_vis(w.n, w.f, device="cuda:0")
    wall, per = time_steps(lambda: xe.correlate(x, vis), calls, 20)
    host = []
    for _ in range(50):
        t0 = time.perf_counter()
        xe.correlate(x, vis)
        torch.cuda.synchronize()
        host.append(time.perf_counter() - t0)
    per_us = sorted(p * 1e6 for p in per)
    host_us = sorted(h * 1e6 for h in host)
    kern, vname, _ = dispatched_kernel(w.n, w.f, w.t)
    return {"workload": w.name, "n": w.n, "f": w.f, "t": w.t, "kernel": kern,
            "device_us_p50": round(per_us[len(per_us) // 2], 2),
            "device_us_mean": round(sum(per_us) / len(per_us), 2),
            "host_call_and_wait_us_p50": round(host_us[len(host_us) // 2], 2),
            "calls_per_s_back_to_back": round(calls / wall, 1)}


def bench_batched(steps: int, warmup: int):
    """64 mixed jobs: one persistent launch (plan) vs one plain launch per job,
    and the plan replayed from a captured HIP graph."""
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics
    from synth import workloads

    specs = workloads.batched_jobs()
    dev = "cuda:0"
    jobs = [(synth.quantized_gaussian(s["f"], s["t"], s["n"], s["sigma"], s["seed"], device=dev),
             xe.new_vis(s["n"], s["f"], device=dev)) for s in specs]
    ops = sum(metrics.effective_ops(s["n"], s["f"], s["t"]) for s in specs)
    plan = xe.Plan(jobs)
    tuned_ms = plan.autotune(reps=2)
    wall_p, per_p = time_steps(plan.run, steps, warmup)
    plain_vis = [xe.new_vis(s["n"], s["f"], device=dev) for s in specs]

    def per_job():
        for (x, _), v in zip(jobs, plain_vis):
            xe.correlate(x, v)

    wall_j, per_j = time_steps(per_job, max(1, steps // 2), 1)
    same = all(bool(torch.equal(v, pv)) for (_, v), pv in zip(jobs, plain_vis))
    plan.capture_graph()
    wall_g, per_g = time_steps(plan.replay, steps, warmup)
    del jobs, plain_vis
    torch.cuda.empty_cache()
    return {
        "workload": "batched", "jobs": len(specs), "effective_ops": ops,
        "plan_tops": round(ops / (sum(per_p) / len(per_p)) / 1e12, 2),
        "graph_tops": round(ops / (sum(per_g) / len(per_g)) / 1e12, 2),
        "per_job_launch_tops": round(ops / (sum(per_j) / len(per_j)) / 1e12, 2),
        "speedup_vs_per_job": round((sum(per_j) / len(per_j)) / (sum(per_p) / len(per_p)), 3),
        "bit_identical_to_per_job": same, "split": plan.split, "tiles": plan.items,
        "autotune_best_ms": round(tuned_ms, 3),
    }


def bench_served(rate_hz: float = 2000.0, frames: int = 2000):
    """Poisson streams of frames through the continuous-batching server.

    The frame mix is N in {256, 2048, 8192} with weights 0.6 / 0.35 / 0.05, F
    uniform in {1, 2, 8}, T = 16384. The HBM budget holds every job's
    accumulator plus 1.5 GiB of frames in flight, so admission defers frames
    when large ones pile up. Runs: the stream at rate_hz (the headline), the
    same frames all at once (closed-loop capacity), a sweep of rates at 25 to
    90 % of that capacity, a uniform mix at rate_hz (overload: about twice
    the capacity is offered), and the same frames as plain per-job launches
    in arrival order (the comparison for aggregate throughput)."""
    import numpy as np
    import torch

    import paper_1503_06203_amd as xe
    import synth
    from paper_1503_06203_amd import metrics, serve
    from synth import workloads

    pools = {}

    def frames_for(n, f):
        if (n, f) not in pools:
            pools[(n, f)] = [synth.quantized_gaussian(f, 16384, n, 2.5,
                                                      seed=5000 + 100 * n + 10 * f + k,
                                                      device="cuda:0") for k in range(2)]
        return pools[(n, f)]

    acc_bytes = sum(metrics.output_bytes(n, f) for n in (256, 2048, 8192) for f in (1, 2, 8))
    budget = acc_bytes + (3 << 29)

    def run(arr, ns, fs):
        stats, acc = serve.run_stream(arr, ns, fs, t, frames_for, hbm_budget=budget,
                                      max_inflight=2)
        del acc
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()}

    arrivals, ns, fs, t = workloads.served_stream(rate_hz=rate_hz, frames=frames)
    out = run(arrivals, ns, fs)
    out.update({"workload": "served", "rate_hz": rate_hz,
                "mix": "N in {256, 2048, 8192} weights 0.6/0.35/0.05, F uniform in {1, 2, 8}, "
                       "T=16384"})
    closed = run(np.zeros_like(arrivals), ns, fs)
    cap = closed["frames_per_s"]
    out["closed_loop"] = {"frames_per_s": cap, "throughput_tops": closed["throughput_tops"],
                          "p50_latency_ms": closed["p50_latency_ms"],
                          "p99_latency_ms": closed["p99_latency_ms"]}
    sweep = []
    for frac in (0.25, 0.5, 0.75, 0.9):
        a, n2, f2, _ = workloads.served_stream(rate_hz=frac * cap, frames=frames // 2, seed=6)
        r = run(a, n2, f2)
        sweep.append({"load": frac, "offered_rate_hz": r["offered_rate_hz"],
                      "throughput_tops": r["throughput_tops"], "frames_per_s": r["frames_per_s"],
                      "p50_latency_ms": r["p50_latency_ms"], "p99_latency_ms": r["p99_latency_ms"]})
    out["rate_sweep"] = sweep
    a, n3, f3, _ = workloads.served_stream(rate_hz=rate_hz, frames=frames // 4, seed=7,
                                           n_weights=(1.0, 1.0, 1.0))
    over = run(a, n3, f3)
    out["overload_uniform_mix"] = {k: over[k] for k in (
        "frames", "completed", "offered_rate_hz", "throughput_tops", "frames_per_s",
        "p50_latency_ms", "p99_latency_ms", "peak_bytes_in_use", "peak_pending_frames")}
    # the same frames, one plain call per frame in arrival order (each job's
    # frames add into its own accumulator), closed loop
    accs = {}
    for n, f in sorted({(int(a), int(b)) for a, b in zip(ns, fs)}):
        accs[(n, f)] = xe.new_vis(n, f, device="cuda:0")
    use = {k: 0 for k in accs}
    calls = []
    for n, f in zip(ns, fs):
        k = (int(n), int(f))
        calls.append((frames_for(*k)[use[k] % 2], accs[k], use[k] * t))
        use[k] += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x, v, held in calls:
        xe.correlate(x, v, accumulate=held > 0, t_prev=held)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ops = sum(metrics.effective_ops(int(n), int(f), t) for n, f in zip(ns, fs))
    out["per_job_plain"] = {"throughput_tops": round(ops / wall / 1e12, 3),
                            "frames_per_s": round(len(calls) / wall, 1)}
    out["served_vs_per_job"] = round(closed["throughput_tops"] / (ops / wall / 1e12), 3)
    del pools, accs, calls
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="large_n",
                    choices=["tiny", "pathfinder", "large_n", "small_n", "batched", "served",
                             "large_n_delayed"])
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-reference", action="store_true",
                    help="also copy 1 GiB device to device (a transfer of known size that "
                         "scales the FETCH_SIZE / WRITE_SIZE hardware counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU and has no multi-GPU path: frequency channels would "
              "shard across GPUs with no exchange, each GPU running this same step on its "
              "share of the channels", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(2)
    from synth import workloads

    def copy_reference():
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload in ("batched", "served"):
        r = bench_batched(args.steps, args.warmup) if args.workload == "batched" else bench_served()
        print(json.dumps(r), flush=True)
        return
    if args.workload == "large_n_delayed":
        # the delayed large-N frame alone (shift kernel, then the rect kernel)
        r = bench_delayed(workloads.LARGE_N, args.steps, args.warmup, main_only=True)
        if args.copy_reference:
            copy_reference()
        print(json.dumps(r), flush=True)
        return

    w = workloads.WORKLOADS[args.workload]
    r = bench_workload(w, args.steps, args.warmup)
    if args.copy_reference:
        copy_reference()
    line = {
        "metric": "effective correlation TOPS (8 ops/complex MAC) + % int8 MFMA peak",
        "value": round(r["value"], 3),
        "unit": "TOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "f": w.f, "t": w.t, "sigma": w.sigma,
                   "common": w.common, "frames": len(w.seeds()),
                   "frame_order": "frames cycle; the first of each cycle overwrites the "
                                  "accumulators, the others add to them",
                   "input": "uint8[F][T][N] 4+4-bit",
                   "output": "int32[F][N(N+1)/2][2]", "parallelism": "single-gpu"},
        "pct_int8_peak": round(100 * r["value"] / PEAK_INT8_TOPS, 2),
        "roofline": mfma_roofline(w, r),
    }
    if w.name == "small_n":
        line["roofline"] = bench_small_n(w, args.steps, args.warmup)["roofline"]
    if not args.no_secondary and w.name == "large_n":
        pw = workloads.PATHFINDER
        pr = bench_workload(pw, 20, 3)
        line["pathfinder"] = {"workload": pw.name, "n": pw.n, "f": pw.f, "t": pw.t,
                              "value": round(pr["value"], 3), "unit": "TOPS",
                              "ms_per_step": round(pr["ms_per_step"], 5),
                              "roofline": mfma_roofline(pw, pr)}
        line["tiny"] = bench_latency(workloads.TINY)
        line["small_n"] = bench_small_n(workloads.SMALL_N, 20, 3)
        line["time_major"] = bench_time_major(pw, 20, 3)
        line["gated"] = bench_gated(pw, 10, 2)
        line["delayed"] = bench_delayed(pw, 10, 2)
        line["large_n_gated"] = bench_gated(w, 5, 1)
        line["large_n_delayed"] = bench_delayed(w, 5, 1)
        line["bf6"] = bench_bf6(pw, 20, 3)
        line["large_n_bf6"] = bench_bf6(w, 10, 2, variant=7)
        line["autotune"] = bench_autotune(w, r)
        line["batched"] = bench_batched(10, 2)
        line["served"] = bench_served()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
