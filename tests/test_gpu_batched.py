"""Batched mode: one persistent launch over a queue of many jobs must give,
bit for bit, what one plain launch per job gives, and what the oracle gives."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1503_06203_amd as xe
import synth
from synth import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


SHAPES = [(4, 1, 100), (64, 2, 333), (128, 1, 1000), (260, 3, 257), (512, 1, 4097), (132, 2, 64),
          (256, 2, 2000), (8, 3, 1)]


def make_jobs(shapes, seed=0):
    jobs = []
    for k, (n, f, t) in enumerate(shapes):
        x = synth.quantized_gaussian(f, t, n, 2.5, seed=seed + 17 * k, device=DEV)
        jobs.append((x, xe.new_vis(n, f, device=DEV)))
    return jobs


def plain(x, prev=None, t_prev=0):
    f, t, n = x.shape
    vis = xe.new_vis(n, f, device=DEV)
    if prev is not None:
        vis.copy_(prev)
    xe.correlate(x, vis, t_prev=t_prev, accumulate=prev is not None)
    return vis


def test_plan_matches_plain_and_oracle():
    jobs = make_jobs(SHAPES)
    plan = xe.Plan(jobs)
    assert plan.items > 0
    plan.run()
    torch.cuda.synchronize()
    for (x, vis) in jobs:
        assert torch.equal(vis, plain(x))
        want = oracle.correlate(x.cpu().numpy())
        assert np.array_equal(vis.cpu().numpy().astype(np.int64), want)
    # counters reset themselves: a second run gives the same sums
    before = [v.clone() for _, v in jobs]
    plan.run()
    torch.cuda.synchronize()
    for b, (_, v) in zip(before, jobs):
        assert torch.equal(b, v)


def test_plan_graph_frames_accumulate():
    shapes = [(256, 2, 1024), (64, 1, 512), (132, 3, 300)]
    frame0 = make_jobs(shapes, seed=1)
    frame1 = [synth.quantized_gaussian(x.shape[0], x.shape[1], x.shape[2], 2.5, seed=900 + k,
                                       device=DEV) for k, (x, _) in enumerate(frame0)]
    plan = xe.Plan(frame0)
    plan.capture_graph()
    for rep in range(3):      # frame 0 replayed (overwrite), with eager work in between
        plan.set_frame([x for x, _ in frame0], accumulate=False)
        plan.replay()
        torch.cuda.synchronize()
        for (x, vis) in frame0:
            assert torch.equal(vis, plain(x)), rep
    plan.set_frame(frame1, accumulate=True)
    plan.replay()
    torch.cuda.synchronize()
    for k, (x, vis) in enumerate(frame0):
        want = plain(frame1[k], prev=plain(x), t_prev=x.shape[1])
        assert torch.equal(vis, want)


def test_plan_long_integration_windows():
    # T above one launch window: atomic partial sums over a zero fill
    x = synth.quantized_gaussian(1, 1_100_000, 8, 2.5, seed=5, device=DEV)
    jobs = [(x, xe.new_vis(8, 1, device=DEV)), (synth.quantized_gaussian(2, 300, 64, 2.5, seed=6,
                                                                         device=DEV),
                                                xe.new_vis(64, 2, device=DEV))]
    jobs[0][1].fill_(12345)
    plan = xe.Plan(jobs)
    plan.run()
    torch.cuda.synchronize()
    for (xx, vis) in jobs:
        assert np.array_equal(vis.cpu().numpy().astype(np.int64), oracle.correlate(xx.cpu().numpy()))


def test_plan_autotune_keeps_results(tmp_path):
    jobs = make_jobs([(256, 4, 4096), (512, 2, 2048), (64, 8, 1000)], seed=3)
    ref = [plain(x) for x, _ in jobs]
    plan = xe.Plan(jobs)
    cache = tmp_path / "tune.txt"
    ms = plan.autotune(reps=2, tune_cache=cache)
    assert ms > 0 and plan.split in (1, 2, 3, 4, 6, 8)
    plan.run()
    torch.cuda.synchronize()
    for r, (_, v) in zip(ref, jobs):
        assert torch.equal(r, v)
    again = xe.Plan(jobs, tune_cache=cache)
    assert again.split == plan.split
    assert os.path.exists(cache)


def test_batched_workload_matches_per_job():
    # the 64-job batched workload (mixed N, F, T), every job bit-identical to its
    # own plain launch; a tile-boundary subset of a few jobs against the oracle
    specs = workloads.batched_jobs()
    jobs = [(synth.quantized_gaussian(s["f"], s["t"], s["n"], s["sigma"], s["seed"], device=DEV),
             xe.new_vis(s["n"], s["f"], device=DEV)) for s in specs]
    plan = xe.Plan(jobs)
    plan.run()
    torch.cuda.synchronize()
    for k, (x, vis) in enumerate(jobs):
        assert torch.equal(vis, plain(x)), k
    # every job against the oracle: all pairs among the elements on both sides
    # of every 128-element edge (every piece boundary) plus a few random ones
    from gpu_helpers import boundary_elements, gather_subset, assert_same
    for k, (x, vis) in enumerate(jobs):
        n = x.shape[2]
        elems = boundary_elements(n, extra=4, seed=k, offsets=(-1, 0))
        sub = x[:, :, torch.as_tensor(elems, device=DEV)].cpu().numpy()
        assert_same(gather_subset(vis, n, elems), oracle.correlate(sub), "job %d" % k)


def test_graph_captured_accumulating_then_overwriting():
    # A plan whose items are split in time combines partial sums with atomic
    # adds, after a zero fill when a job overwrites. Captured while the jobs
    # accumulate, the graph must still zero-fill once set_frame switches them
    # to overwriting (the fill kernel reads each job's flag on the device).
    shapes = [(256, 2, 2048), (512, 1, 1500)]
    jobs = make_jobs(shapes, seed=7)
    plan = xe.Plan(jobs)
    plan.autotune(reps=1)                      # overwriting jobs: allowed
    frame1 = [synth.quantized_gaussian(x.shape[0], x.shape[1], x.shape[2], 2.5, seed=70 + k,
                                       device=DEV) for k, (x, _) in enumerate(jobs)]
    plan.set_frame(frame1, accumulate=True)
    # (with no time split chosen there are no atomic adds, and the replays
    # below still check that the graph follows the accumulate flags)
    plan.capture_graph()
    plan.replay()                              # frame 0 + frame 1
    torch.cuda.synchronize()
    plan.set_frame(frame1, accumulate=False)   # overwrite with frame 1 alone
    for rep in range(3):
        for (_, v) in jobs:
            v.fill_(-12345)                    # stale sums the fill must clear
        plan.replay()
        torch.cuda.synchronize()
        for k, (_, v) in enumerate(jobs):
            want = oracle.correlate(frame1[k].cpu().numpy())
            assert np.array_equal(v.cpu().numpy().astype(np.int64), want), (rep, k)


def test_forced_split_graph_zero_fill(tmp_path):
    # the same with a tuned split of 4 read from a cache file (no autotune run)
    shapes = [(256, 2, 2048), (512, 1, 1500)]
    jobs = make_jobs(shapes, seed=8)
    key = "plan" + "".join(":%dx%dx%d" % (x.shape[2], x.shape[0], x.shape[1]) for x, _ in jobs)
    cache = tmp_path / "tune.txt"
    cache.write_text(key + " 4\n")
    plan = xe.Plan(jobs, tune_cache=cache)
    assert plan.split == 4
    plan.set_frame(None, accumulate=True)
    plan.capture_graph()
    plan.set_frame(None, accumulate=False)
    for (_, v) in jobs:
        v.fill_(777)
    plan.replay()
    torch.cuda.synchronize()
    for (x, v) in jobs:
        assert np.array_equal(v.cpu().numpy().astype(np.int64), oracle.correlate(x.cpu().numpy()))


def test_autotune_refuses_accumulating_plan():
    shapes = [(256, 2, 512), (64, 1, 300)]
    jobs = make_jobs(shapes, seed=9)
    plan = xe.Plan(jobs)
    plan.run()
    torch.cuda.synchronize()
    before = [v.clone() for _, v in jobs]
    plan.set_frame(None, accumulate=True)
    with pytest.raises(xe.XengError) as e:
        plan.autotune(reps=2)
    assert e.value.status == -1
    torch.cuda.synchronize()
    for b, (_, v) in zip(before, jobs):
        assert torch.equal(b, v)               # nothing ran
    plan.run()                                 # the accumulating frame, once
    torch.cuda.synchronize()
    for b, (x, v) in zip(before, jobs):
        assert torch.equal(v, plain(x, prev=b, t_prev=x.shape[1]))
