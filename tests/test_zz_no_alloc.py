"""The allocation-free plan run (xeng_plan_run_static): through the C ABI it
must give, bit for bit, what xeng_plan_run gives with a caller workspace, on
consecutive calls that share the library's static device array (the second
with a smaller plan than the first), and what the oracle gives."""
import numpy as np
import pytest
import torch

import oracle
import paper_1503_06203_amd as xe
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def make_jobs(shapes, seed):
    jobs = []
    for k, (n, f, t) in enumerate(shapes):
        x = synth.quantized_gaussian(f, t, n, 2.5, seed=seed + 31 * k, device=DEV)
        jobs.append((x, xe.new_vis(n, f, device=DEV)))
    return jobs


def spoil(jobs):
    for _, vis in jobs:
        vis.fill_(0x5A5A5A5A)


def check_static_equals_workspace_run(plan, jobs, oracle_jobs=()):
    plan.run()
    torch.cuda.synchronize()
    want = [vis.clone() for _, vis in jobs]
    spoil(jobs)
    plan.run_static()
    torch.cuda.synchronize()
    for k, ((x, vis), w) in enumerate(zip(jobs, want)):
        assert torch.equal(vis, w), "job %d differs from the workspace run" % k
    for k in oracle_jobs:
        x, vis = jobs[k]
        got = vis.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, oracle.correlate(x.cpu().numpy())), "job %d vs oracle" % k


def test_static_run_twice_second_smaller(tmp_path):
    # first plan: large and small pieces, time split 2 from a tune cache so the
    # zero fill and the atomic adds also run out of the static array
    shapes_a = [(2048, 2, 1000), (512, 3, 777), (260, 1, 4097), (64, 4, 3000), (4, 1, 65)]
    jobs_a = make_jobs(shapes_a, seed=11)
    key = "plan" + "".join(":%dx%dx%d" % s for s in shapes_a)
    cache = tmp_path / "tune.txt"
    cache.write_text("%s 2\n" % key)
    plan_a = xe.Plan(jobs_a, tune_cache=str(cache))
    assert plan_a.split == 2
    check_static_equals_workspace_run(plan_a, jobs_a, oracle_jobs=(1, 2, 3, 4))
    # second plan, smaller than the first: no split, fewer and smaller jobs; the
    # array still holds the first plan's image and counters
    shapes_b = [(256, 2, 300), (68, 1, 129)]
    jobs_b = make_jobs(shapes_b, seed=23)
    plan_b = xe.Plan(jobs_b)
    assert plan_b.split == 1 and plan_b.items < plan_a.items
    check_static_equals_workspace_run(plan_b, jobs_b, oracle_jobs=(0, 1))
    # and the first plan again after the second
    check_static_equals_workspace_run(plan_a, jobs_a)


def test_static_run_without_workspace_frames():
    """A plan built with no device allocation at all, fed two frames through
    set_frame without a workspace: overwrite, then accumulate."""
    shapes = [(512, 2, 640), (128, 3, 200)]
    frame0 = make_jobs(shapes, seed=41)
    frame1 = [synth.quantized_gaussian(x.shape[0], x.shape[1], x.shape[2], 2.5, seed=77 + k,
                                       device=DEV) for k, (x, _) in enumerate(frame0)]
    plan = xe.Plan(frame0, workspace=False)
    assert plan.workspace is None
    with pytest.raises(xe.XengError):
        plan.run()
    plan.run_static()
    torch.cuda.synchronize()
    for x, vis in frame0:
        assert np.array_equal(vis.cpu().numpy().astype(np.int64), oracle.correlate(x.cpu().numpy()))
    plan.set_frame(frame1, accumulate=True)
    plan.run_static()
    torch.cuda.synchronize()
    for (x0, vis), x1 in zip(frame0, frame1):
        both = np.concatenate([x0.cpu().numpy(), x1.cpu().numpy()], axis=1)
        assert np.array_equal(vis.cpu().numpy().astype(np.int64), oracle.correlate(both))
    plan.set_frame(None, accumulate=False)
    spoil(frame0)
    plan.run_static()
    torch.cuda.synchronize()
    for x1, (_, vis) in zip(frame1, frame0):
        assert np.array_equal(vis.cpu().numpy().astype(np.int64), oracle.correlate(x1.cpu().numpy()))
