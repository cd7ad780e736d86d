"""Delay compensation (per-element integer sample delays applied while the
samples are staged) against the oracle's gather-then-correlate."""
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


def delayed(x_dev, delays, prev=None, t_prev=0):
    import paper_1503_06203_amd as xe
    f, _, n = x_dev.shape
    vis = torch.zeros((f, xe.vis_entries(n), 2), dtype=torch.int32, device=DEV)
    if prev is not None:
        vis.copy_(prev)
    xe.correlate_delayed(x_dev, vis, delays, t_prev=t_prev, accumulate=prev is not None)
    torch.cuda.synchronize()
    return vis


@pytest.mark.parametrize("f,t,n,dmax", [(3, 1024, 256, 300), (2, 64, 5, 7), (4, 512, 130, 64),
                                        (1, 16384, 256, 1000), (2, 2048, 96, 1)])
def test_delayed_matches_oracle(f, t, n, dmax):
    print("delayed f=%d t=%d n=%d dmax=%d" % (f, t, n, dmax), flush=True)
    rng = np.random.default_rng(f + t + n + dmax)
    delays = rng.integers(0, dmax + 1, n)
    delays[0] = dmax
    x = synth.quantized_gaussian(f, t + dmax, n, 2.5, seed=f * 31 + n)
    got = delayed(x.to(DEV), delays)
    assert_same(got, oracle.correlate_delayed(x.numpy(), delays), "delayed")


def test_delayed_zero_equals_plain():
    import paper_1503_06203_amd as xe
    x = synth.uniform_bytes(3, 1024, 256, seed=41).to(DEV)
    got = delayed(x, np.zeros(256, dtype=np.int32))
    plain = xe.correlate(x, xe.new_vis(256, 3))
    torch.cuda.synchronize()
    assert torch.equal(got, plain)


def test_delayed_largest_delay_and_accumulate():
    f, t, n = 1, 128, 64
    delays = np.zeros(n, dtype=np.int32)
    delays[::7] = 65535
    x = synth.uniform_bytes(f, t + 65535, n, seed=42)
    first = delayed(x.to(DEV), delays)
    want = oracle.correlate_delayed(x.numpy(), delays)
    assert_same(first, want, "max delay")
    twice = delayed(x.to(DEV), delays, prev=first, t_prev=t)
    assert_same(twice, 2 * want, "accumulated")


def test_delayed_errors():
    import paper_1503_06203_amd as xe
    vis = torch.zeros((1, xe.vis_entries(16), 2), dtype=torch.int32, device=DEV)
    with pytest.raises(xe.XengError):                       # t = 100 - 4 is not a multiple of 64
        xe.correlate_delayed(torch.zeros((1, 100, 16), dtype=torch.uint8, device=DEV), vis,
                             [4] + [0] * 15)
    with pytest.raises(xe.XengError):                       # negative delay
        xe.correlate_delayed(torch.zeros((1, 64, 16), dtype=torch.uint8, device=DEV), vis,
                             [-1] + [0] * 15)
    big = torch.zeros((1, 64, 300), dtype=torch.uint8, device=DEV)
    with pytest.raises(xe.XengError):                       # beyond the triangle kernel
        xe.correlate_delayed(big, torch.zeros((1, xe.vis_entries(300), 2), dtype=torch.int32,
                                              device=DEV), [0] * 300)
    with pytest.raises(xe.XengError):                       # range guard
        xe.correlate_delayed(torch.zeros((1, 64, 16), dtype=torch.uint8, device=DEV), vis,
                             [0] * 16, t_prev=xe.MAX_SAMPLES, accumulate=True)


# Delay spreads up to 128 samples with n % 4 == 0 take the window form (the
# rows of a stage loaded whole into an LDS ring, gathered there); the cases
# above with larger spreads or odd n take the per-byte gather form.
@pytest.mark.parametrize("f,t,n,lo,hi", [(3, 1024, 256, 0, 128), (2, 640, 64, 37, 137),
                                         (1, 16384, 256, 0, 100), (5, 192, 4, 10, 11),
                                         (2, 4096, 132, 64, 191)])
def test_delayed_window_form(f, t, n, lo, hi):
    print("window f=%d t=%d n=%d delays %d..%d" % (f, t, n, lo, hi), flush=True)
    rng = np.random.default_rng(f * 7 + n + hi)
    delays = rng.integers(lo, hi + 1, n)
    delays[0], delays[-1] = lo, hi
    dmax = hi
    x = synth.quantized_gaussian(f, t + dmax, n, 2.5, seed=f * 31 + n + 5)
    got = delayed(x.to(DEV), delays)
    assert_same(got, oracle.correlate_delayed(x.numpy(), delays), "window")


def test_delayed_window_accumulate_matches_gather_form():
    # the same delays once within the window spread and once with one more
    # element far outside it (gather form): both equal the oracle
    f, t, n = 2, 2048, 128
    rng = np.random.default_rng(3)
    near = rng.integers(0, 60, n)
    x = synth.uniform_bytes(f, t + 400, n, seed=77)
    xn = x[:, :t + int(near.max())].contiguous()       # [F][T + D][N], D = the largest delay
    first = delayed(xn.to(DEV), near)
    twice = delayed(xn.to(DEV), near, prev=first, t_prev=t)
    want = oracle.correlate_delayed(xn.numpy(), near)
    assert_same(twice, 2 * want, "window accumulate")
    far = near.copy()
    far[5] = 400
    got = delayed(x.to(DEV), far)
    assert_same(got, oracle.correlate_delayed(x.numpy(), far), "gather form")



@pytest.mark.parametrize("n,d,dmax", [(256, 17, 40), (64, 40, 40), (96, 0, 9)])
def test_delayed_common_delay(n, d, dmax):
    # one delay for every element: the shifted-window plain correlation, with
    # max_delay above the common delay (the C-ABI allows it)
    import ctypes

    import paper_1503_06203_amd as xe
    print("common delay n=%d d=%d max_delay=%d" % (n, d, dmax), flush=True)
    f, t = 2, 512
    delays = np.full(n, d, dtype=np.int32)
    x = synth.quantized_gaussian(f, t + dmax, n, 2.5, seed=n + d)
    xd = x.to(DEV)
    vis = torch.zeros((f, xe.vis_entries(n), 2), dtype=torch.int32, device=DEV)
    for acc in (0, 1):
        xe.check(xe.lib().xeng_correlate_delayed(
            xd.data_ptr(), vis.data_ptr(), n, f, t, delays.ctypes.data_as(ctypes.c_void_p), dmax,
            t if acc else 0, acc, xe._stream_ptr(None)))
    torch.cuda.synchronize()
    want = oracle.correlate(np.ascontiguousarray(x.numpy()[:, dmax - d: dmax - d + t, :]))
    assert_same(vis, 2 * want, "common delay, accumulated")


def _unaligned(x):
    # a device copy of x that starts one byte into its allocation
    flat = torch.empty(x.numel() + 1, dtype=torch.uint8, device=DEV)
    flat[1:].copy_(x.reshape(-1).to(DEV))
    view = flat[1:].view(*x.shape)
    assert view.data_ptr() % 4 == 1
    return view


def test_delayed_unaligned_input():
    # unaligned input: every element is gathered bytewise
    f, t, n, dmax = 2, 256, 64, 20
    print("unaligned delayed f=%d t=%d n=%d" % (f, t, n), flush=True)
    rng = np.random.default_rng(77)
    delays = rng.integers(0, dmax + 1, n)
    delays[0] = dmax
    x = synth.quantized_gaussian(f, t + dmax, n, 2.5, seed=78)
    got = delayed(_unaligned(x), delays)
    assert_same(got, oracle.correlate_delayed(x.numpy(), delays), "unaligned delayed")
    common = np.full(n, 5, dtype=np.int32)
    x5 = synth.quantized_gaussian(f, t + 5, n, 2.5, seed=79)
    got5 = delayed(_unaligned(x5), common)
    assert_same(got5, oracle.correlate_delayed(x5.numpy(), common), "unaligned common delay")
