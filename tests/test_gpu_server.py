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


def test_served_shapes_alone_equals_mix_and_oracle():
    # The served workload's job shapes: N in {256, 2048, 8192}, F in {1, 2, 8},
    # T = 16384 per frame, sigma 2.5. Frames of every job are interleaved and
    # served with continuous batching; each job's sums must equal its frames
    # run alone (tolerance 0) and the oracle: in full for an N=256 job and one
    # channel of an N=2048 job, and for the N=8192, F=1 job on every pair of a
    # tile-boundary element subset plus five whole rows.
    from gpu_helpers import boundary_elements, gather_subset
    t = 16384
    jobs = {"a": (256, 8, 3), "b": (2048, 2, 2), "c": (8192, 1, 2), "d": (8192, 8, 1),
            "e": (2048, 8, 1), "f": (256, 1, 2)}
    frames = {k: [synth.quantized_gaussian(f, t, n, 2.5, seed=500 + 10 * i + j, device=DEV)
                  for j in range(nf)]
              for i, (k, (n, f, nf)) in enumerate(jobs.items())}
    srv = xe.Server(hbm_budget=64 << 30, max_inflight=2)
    acc = {k: xe.new_vis(n, f, device=DEV) for k, (n, f, _) in jobs.items()}
    ids = {k: srv.open_job(jobs[k][0], jobs[k][1], acc[k]) for k in jobs}
    order = [(k, j) for j in range(3) for k in jobs if j < jobs[k][2]]
    tickets = []
    for i, (k, j) in enumerate(order):
        tickets.append(srv.submit(ids[k], frames[k][j]))
        if i % 2 == 1:
            srv.step()
    srv.drain()
    for tk in tickets:
        done, lat = srv.poll(tk)
        assert done and lat >= 0.0
    for k in jobs:
        assert torch.equal(acc[k], alone(frames[k])), k
    # N=256, F=8: every entry of every channel
    xa = torch.cat(frames["a"], dim=1).cpu().numpy()
    assert np.array_equal(acc["a"].cpu().numpy().astype(np.int64), oracle.correlate(xa))
    # N=2048, F=2: every entry of channel 1
    xb = torch.cat([x[1:2] for x in frames["b"]], dim=1).cpu().numpy()
    assert np.array_equal(acc["b"][1:2].cpu().numpy().astype(np.int64), oracle.correlate(xb))
    # N=8192, F=1: all pairs among elements around every 128/256 edge
    n = 8192
    xc = torch.cat(frames["c"], dim=1)
    elems = boundary_elements(n, tile=128, extra=16, offsets=(-1, 0))
    sub = xc[:, :, torch.as_tensor(elems, device=DEV)].cpu().numpy()
    assert np.array_equal(gather_subset(acc["c"], n, elems), oracle.correlate(sub))
    # ... and whole rows i (every j >= i)
    xcc = xc.cpu().numpy()
    for i in (0, 255, 256, 4095, n - 129):
        j = np.arange(i, n)
        fij = np.stack([np.zeros_like(j), np.full_like(j, i), j], axis=1)
        k0 = i * (2 * n - i + 1) // 2
        got = acc["c"][0, k0:k0 + len(j)].cpu().numpy().astype(np.int64)
        assert np.array_equal(got, oracle.entries(xcc, fij)), i
    for k in jobs:
        srv.close_job(ids[k])
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


def test_many_frames_of_a_job_in_one_step():
    # Every frame is submitted before the first step: after a job's first frame
    # (which overwrites its accumulator, alone in its step) a step takes up to
    # 16 of its pending frames at once, each added into the sums with int32
    # atomic adds. The sums must equal the frames run alone, in order, and the
    # oracle; the budget admits only some of the frames at a time, so later
    # frames of a job wait behind earlier ones.
    shapes = {"a": (260, 2, 300), "b": (64, 3, 129), "c": (512, 1, 1000)}
    nframes = {"a": 21, "b": 9, "c": 5}
    frames = {k: [synth.quantized_gaussian(f, t, n, 2.5, seed=900 + 50 * i + j, device=DEV)
                  for j in range(nframes[k])]
              for i, (k, (n, f, t)) in enumerate(shapes.items())}
    acc_bytes = sum(f * (n * (n + 1) // 2) * 8 for n, f, _ in shapes.values())
    frame_bytes = max(n * f * t for n, f, t in shapes.values())
    srv = xe.Server(hbm_budget=acc_bytes + 6 * frame_bytes, max_inflight=2)
    acc = {k: xe.new_vis(n, f, device=DEV) for k, (n, f, t) in shapes.items()}
    for v in acc.values():
        v.fill_(-77)                       # the first frame of each job overwrites
    ids = {k: srv.open_job(shapes[k][0], shapes[k][1], acc[k]) for k in shapes}
    tickets = [srv.submit(ids[k], x) for k in shapes for x in frames[k]]
    srv.drain()
    for tk in tickets:
        assert srv.poll(tk)[0]
    for k in shapes:
        assert torch.equal(acc[k], alone(frames[k])), k
        x = torch.cat(frames[k], dim=1).cpu().numpy()
        assert np.array_equal(acc[k].cpu().numpy().astype(np.int64), oracle.correlate(x)), k
    srv.close()
