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


def _c_delayed(x, vis, delays, dmax, t):
    """xeng_correlate_delayed (the fused entry point, no workspace) directly."""
    import ctypes

    import paper_1503_06203_amd as xe
    d = np.ascontiguousarray(np.asarray(delays, dtype=np.int32))
    return xe.lib().xeng_correlate_delayed(x.data_ptr(), vis.data_ptr(), x.shape[2], x.shape[0],
                                           t, d.ctypes.data_as(ctypes.c_void_p), dmax, 0, 0,
                                           xe._stream_ptr(None))


def test_delayed_errors():
    import paper_1503_06203_amd as xe
    EINVAL = -1
    vis = torch.zeros((1, xe.vis_entries(16), 2), dtype=torch.int32, device=DEV)
    # the fused entry point: t = 96 is not a multiple of 64, n = 300 is above 256
    x100 = torch.zeros((1, 100, 16), dtype=torch.uint8, device=DEV)
    assert _c_delayed(x100, vis, [4] + [0] * 15, 4, 96) == EINVAL
    assert b"xeng_correlate_delayed_ws" in xe.lib().xeng_last_error()
    big = torch.zeros((1, 64, 300), dtype=torch.uint8, device=DEV)
    vbig = torch.zeros((1, xe.vis_entries(300), 2), dtype=torch.int32, device=DEV)
    assert _c_delayed(big, vbig, [0] * 300, 0, 64) == EINVAL
    with pytest.raises(xe.XengError):                       # negative delay
        xe.correlate_delayed(torch.zeros((1, 64, 16), dtype=torch.uint8, device=DEV), vis,
                             [-1] + [0] * 15)
    with pytest.raises(xe.XengError):                       # range guard
        xe.correlate_delayed(torch.zeros((1, 64, 16), dtype=torch.uint8, device=DEV), vis,
                             [0] * 16, t_prev=xe.MAX_SAMPLES, accumulate=True)
    # the workspace form (unequal delays, so the samples are shifted): a
    # workspace below f * n * min(t, 128) bytes, t = 64 here
    big1 = torch.zeros((1, 65, 300), dtype=torch.uint8, device=DEV)
    uneq = [1] + [0] * 299
    with pytest.raises(xe.XengError) as e:
        xe.correlate_delayed(big1, vbig, uneq,
                             workspace=torch.empty(300 * 63, dtype=torch.uint8, device=DEV))
    assert "too small" in str(e.value)
    # a workspace that overlaps the input
    x2 = torch.zeros((1, 65 + 1024, 300), dtype=torch.uint8, device=DEV)
    with pytest.raises(xe.XengError) as e:
        xe.correlate_delayed(x2[:, :65], vbig, uneq, workspace=x2.reshape(-1)[1000:])
    assert "overlaps" in str(e.value)


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


# Arrays above 256 elements, and frames that are not whole 64-sample stages,
# run shift-then-correlate: windows of frame samples are written delay-aligned
# into a workspace (staged through LDS when a 256-element block's delays
# differ by at most 128 samples, else byte by byte) and correlated by the
# plain kernels. Spreads 0, 1, 128 and 300; tails of both piece kinds; the
# full-CHIME array size. One delay common to all elements of an aligned input
# (the first case) is the plain correlation of a shifted window, read in place.
@pytest.mark.parametrize("f,t,n,lo,hi", [(2, 1024, 260, 5, 5), (2, 1000, 516, 0, 1),
                                         (1, 2048, 1024, 0, 128), (2, 4096, 2048, 0, 128),
                                         (1, 640, 516, 0, 300), (3, 100, 64, 3, 90),
                                         (1, 129, 2048, 0, 64), (2, 300, 261, 4, 4),
                                         (1, 2300, 1040, 10, 110)])
def test_delayed_shift_form(f, t, n, lo, hi):
    print("shift form f=%d t=%d n=%d delays %d..%d" % (f, t, n, lo, hi), flush=True)
    rng = np.random.default_rng(f * 11 + n + hi + t)
    delays = rng.integers(lo, hi + 1, n)
    delays[0], delays[-1] = lo, hi
    x = synth.quantized_gaussian(f, t + hi, n, 2.5, seed=f * 37 + n + hi)
    got = delayed(x.to(DEV), delays)
    assert_same(got, oracle.correlate_delayed(x.numpy(), delays), "shift form")


def test_delayed_shift_form_windows_and_accumulate():
    # a workspace of three 128-sample windows: 1000 samples run as 384 + 384 +
    # 232, the same sums as one pass; then accumulated onto held sums
    import paper_1503_06203_amd as xe
    f, t, n, dmax = 2, 1000, 388, 200
    rng = np.random.default_rng(5)
    delays = rng.integers(0, dmax + 1, n)
    delays[7] = dmax
    x = synth.quantized_gaussian(f, t + dmax, n, 2.5, seed=55)
    xd = x.to(DEV)
    want = oracle.correlate_delayed(x.numpy(), delays)
    small = torch.empty(f * n * 128 * 3 + 5, dtype=torch.uint8, device=DEV)
    vis = torch.full((f, xe.vis_entries(n), 2), -9, dtype=torch.int32, device=DEV)
    xe.correlate_delayed(xd, vis, delays, workspace=small)
    torch.cuda.synchronize()
    assert_same(vis, want, "windowed")
    xe.correlate_delayed(xd, vis, delays, t_prev=t, accumulate=True)
    torch.cuda.synchronize()
    assert_same(vis, 2 * want, "windowed, accumulated")


def test_delayed_shift_form_unaligned():
    # n % 4 != 0 and a misaligned input: bytewise shift, general kernel
    for n, t, dmax in ((261, 300, 40), (300, 257, 129)):
        print("unaligned shift n=%d t=%d" % (n, t), flush=True)
        rng = np.random.default_rng(n)
        delays = rng.integers(0, dmax + 1, n)
        delays[1] = dmax
        x = synth.quantized_gaussian(2, t + dmax, n, 2.5, seed=n + 1)
        got = delayed(_unaligned(x), delays)
        assert_same(got, oracle.correlate_delayed(x.numpy(), delays), "unaligned shift")
