"""Serving mode: frames streamed into device-resident accumulators with
continuous batching give, for every job, exactly the sums of that job's frames
run alone."""
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


def alone(frames):
    f, t, n = frames[0].shape
    vis = xe.new_vis(n, f, device=DEV)
    held = 0
    for k, x in enumerate(frames):
        xe.correlate(x, vis, t_prev=held, accumulate=k > 0)
        held += x.shape[1]
    torch.cuda.synchronize()
    return vis


def test_alone_equals_mix():
    shapes = {"a": (256, 2, 512), "b": (64, 1, 300), "c": (132, 3, 257), "d": (512, 1, 1024)}
    nframes = {"a": 4, "b": 6, "c": 3, "d": 2}
    frames = {k: [synth.quantized_gaussian(f, t, n, 2.5, seed=100 * i + j, device=DEV)
                  for j in range(nframes[k])]
              for i, (k, (n, f, t)) in enumerate(shapes.items())}
    srv = xe.Server(hbm_budget=8 << 30, max_inflight=2)
    acc = {k: xe.new_vis(n, f, device=DEV) for k, (n, f, t) in shapes.items()}
    ids = {k: srv.open_job(shapes[k][0], shapes[k][1], acc[k]) for k in shapes}
    tickets = []
    # interleave submissions with steps: frames arrive while others run
    order = [(k, j) for j in range(max(nframes.values())) for k in shapes if j < nframes[k]]
    for i, (k, j) in enumerate(order):
        tickets.append(srv.submit(ids[k], frames[k][j]))
        if i % 3 == 2:
            srv.step()
    srv.drain()
    for tk in tickets:
        done, lat = srv.poll(tk)
        assert done and lat >= 0.0
    for k in shapes:
        assert torch.equal(acc[k], alone(frames[k])), k
    x = torch.cat(frames["c"], dim=1).cpu().numpy()
    assert np.array_equal(acc["c"].cpu().numpy().astype(np.int64), oracle.correlate(x))
    for k in shapes:
        srv.close_job(ids[k])
    assert srv.stats()["open_jobs"] == 0
    srv.close()


def test_admission_and_backpressure():
    n, f = 256, 2
    acc_bytes = f * n * (n + 1) // 2 * 8
    srv = xe.Server(hbm_budget=acc_bytes + 100, max_inflight=1)
    v1 = xe.new_vis(n, f, device=DEV)
    j1 = srv.open_job(n, f, v1)
    with pytest.raises(xe.XengError) as e:
        srv.open_job(n, f, xe.new_vis(n, f, device=DEV))        # accumulator does not fit
    assert e.value.status == -5
    x = synth.quantized_gaussian(f, 64, n, 2.5, seed=1, device=DEV)
    tk = srv.submit(j1, x)                    # frame bytes exceed what is left: must wait
    assert srv.step() == 0
    with pytest.raises(xe.XengError):
        srv.close_job(j1)                      # frame still queued
    with pytest.raises(xe.XengError) as e:
        srv.drain()                            # can never be admitted under this budget
    assert e.value.status == -5
    srv.close()
    # a budget that fits one frame at a time still serves every frame in order
    srv = xe.Server(hbm_budget=acc_bytes + f * 64 * n, max_inflight=2)
    v = xe.new_vis(n, f, device=DEV)
    j = srv.open_job(n, f, v)
    xs = [synth.quantized_gaussian(f, 64, n, 2.5, seed=10 + k, device=DEV) for k in range(5)]
    for xx in xs:
        srv.submit(j, xx)
    srv.drain()
    assert torch.equal(v, alone(xs))
    srv.close()


def test_range_guard_and_bad_frames():
    srv = xe.Server(hbm_budget=1 << 30, max_inflight=1)
    n, f = 8, 1
    j = srv.open_job(n, f, xe.new_vis(n, f, device=DEV))
    with pytest.raises(xe.XengError):
        srv.open_job(6, 1, xe.new_vis(6, 1, device=DEV))     # n % 4 != 0
    with pytest.raises(xe.XengError):
        srv.submit(j + 99, torch.zeros((1, 4, n), dtype=torch.uint8, device=DEV))   # unknown job
    srv.close()
