"""Gated correlation (one accumulator set per gate bin) against the oracle's
per-gate sums."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


from gpu_helpers import assert_same  # noqa: E402


def gated(x_dev, sched, block, gates, prev=None, t_prev=None):
    import paper_1503_06203_amd as xe
    f, t, n = x_dev.shape
    vis = torch.zeros((gates, f, xe.vis_entries(n), 2), dtype=torch.int32, device=DEV)
    if prev is not None:
        vis.copy_(prev)
    xe.correlate_gated(x_dev, vis, sched, block, t_prev=t_prev, accumulate=prev is not None)
    torch.cuda.synchronize()
    return vis


@pytest.mark.parametrize("f,t,n,block,gates", [(2, 1000, 64, 64, 3), (1, 777, 256, 100, 2),
                                               (3, 4096, 384, 512, 4), (2, 130, 8, 7, 2)])
def test_gated_matches_oracle(f, t, n, block, gates):
    x = synth.quantized_gaussian(f, t, n, 2.5, seed=f * 17 + t + n + block)
    nb = (t + block - 1) // block
    rng = np.random.default_rng(t + block)
    sched = rng.integers(0, gates, nb).astype(np.uint8)
    sched[rng.integers(0, nb)] = 0xFF                      # one flagged block
    got = gated(x.to(DEV), sched, block, gates)
    assert_same(got, oracle.correlate_gated(x.numpy(), sched, block, gates), "gated")


def test_gated_accumulate_and_empty_gate():
    f, t, n, block = 2, 512, 128, 64
    x = synth.uniform_bytes(f, t, n, seed=31)
    sched = np.array([0, 0, 1, 1, 0, 0, 1, 1], dtype=np.uint8)
    first = gated(x.to(DEV), sched, block, 3)
    assert not first[2].any()                               # gate 2 received nothing: zero
    twice = gated(x.to(DEV), sched, block, 3, prev=first, t_prev=[256, 256, 0])
    want = oracle.correlate_gated(x.numpy(), sched, block, 3)
    assert_same(twice, 2 * want, "accumulated")


def test_gated_errors():
    import paper_1503_06203_amd as xe
    x = torch.zeros((1, 100, 16), dtype=torch.uint8, device=DEV)
    vis = torch.zeros((2, 1, xe.vis_entries(16), 2), dtype=torch.int32, device=DEV)
    with pytest.raises(xe.XengError):
        xe.correlate_gated(x, vis, [0, 5], 50)               # gate index out of range
    with pytest.raises(xe.XengError):
        xe.correlate_gated(x, vis, [0, 1], 50, t_prev=[xe.MAX_SAMPLES, 0], accumulate=True)


# With N <= 256 all runs of one gate go to the triangle kernel in one launch
# (at most 32 runs per launch): many short runs (several launches per gate),
# runs not aligned to the 64-sample stages, and one long gate on one channel
# (split along time, atomic adds).
@pytest.mark.parametrize("f,t,n,block,gates", [(2, 4096, 64, 8, 2), (1, 16384, 128, 1024, 2),
                                               (3, 2000, 256, 37, 3)])
def test_gated_segments(f, t, n, block, gates):
    print("gated segments f=%d t=%d n=%d block=%d gates=%d" % (f, t, n, block, gates), flush=True)
    x = synth.quantized_gaussian(f, t, n, 2.5, seed=t + n + block)
    nb = (t + block - 1) // block
    sched = (np.arange(nb) % gates).astype(np.uint8)
    if block == 1024:
        sched[:] = 0
        sched[3] = 1
    got = gated(x.to(DEV), sched, block, gates)
    assert_same(got, oracle.correlate_gated(x.numpy(), sched, block, gates), "gated segments")


# Above 256 elements the runs of one gate go to the kernel of diagonal squares
# and 128 x 256 tiles in one launch per gate (at most 32 runs per launch):
# tails of both piece kinds (N = 260, 516), many short runs, runs off the
# 64-sample stage grid, a long gate split along time, and the full-CHIME
# array size.
@pytest.mark.parametrize("f,t,n,block,gates", [(2, 4096, 260, 8, 2), (1, 16384, 512, 1024, 2),
                                               (3, 2000, 516, 37, 3), (2, 8192, 2048, 1024, 2)])
def test_gated_segments_large_n(f, t, n, block, gates):
    print("gated segments f=%d t=%d n=%d block=%d gates=%d" % (f, t, n, block, gates), flush=True)
    x = synth.quantized_gaussian(f, t, n, 2.5, seed=t + n + block + 5)
    nb = (t + block - 1) // block
    sched = (np.arange(nb) % gates).astype(np.uint8)
    if block == 1024:
        sched[:] = 0
        sched[3] = 1
        sched[-1] = 0xFF
    got = gated(x.to(DEV), sched, block, gates)
    assert_same(got, oracle.correlate_gated(x.numpy(), sched, block, gates), "gated segments")
    if n == 2048:
        # gates partition the samples: their sums add up to the plain correlation
        import paper_1503_06203_amd as xe
        keep = np.repeat(sched != 0xFF, block)[:t]
        xs = x[:, torch.as_tensor(keep)].contiguous().to(DEV)
        plain = xe.new_vis(n, f, device=DEV)
        xe.correlate(xs, plain)
        torch.cuda.synchronize()
        assert torch.equal(got.sum(dim=0, dtype=torch.int64).to(torch.int32), plain)
