"""Bit-exact parity of the HIP path against the CPU oracle (tolerance 0).

Every input is seeded and synthetic. Small shapes are checked in full; the
full-size workloads are checked on every entry among a set of elements that
straddles every tile boundary (sub-matrix property: V_ij depends only on
elements i and j), plus full oracle channels where that is cheap."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


from gpu_helpers import (assert_same, boundary_elements, gather_subset, gpu_correlate,  # noqa: E402
                         subset_reference)


def full_check(x_cpu, **kw):
    vis = gpu_correlate(x_cpu.to(DEV), **kw)
    assert_same(vis, oracle.correlate(x_cpu.numpy()), str(tuple(x_cpu.shape)))


def test_tiny_workload():
    w = workloads.TINY
    x = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seed)
    full_check(x)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 17, 31, 33, 64, 100, 127, 128, 129, 255, 256, 257])
def test_element_tails(n):
    x = synth.uniform_bytes(2, 97, n, seed=n)
    full_check(x)


@pytest.mark.parametrize("t", [1, 2, 15, 16, 17, 31, 33, 63, 64, 65, 127, 129, 4097])
def test_time_tails(t):
    x = synth.quantized_gaussian(1, t, 160, 3.0, seed=t)
    full_check(x)


def test_empty_time_axis_zero_fills_and_accumulate_is_noop():
    import paper_1503_06203_amd as xe
    x = torch.zeros((2, 0, 40), dtype=torch.uint8, device=DEV)
    vis = torch.full((2, xe.vis_entries(40), 2), 7, dtype=torch.int32, device=DEV)
    xe.correlate(x, vis, accumulate=True, t_prev=3)
    torch.cuda.synchronize()
    assert (vis == 7).all()
    xe.correlate(x, vis)
    torch.cuda.synchronize()
    assert (vis == 0).all()


@pytest.mark.parametrize("byte,re", [(0x00, 128), (0xFF, 98), (0x88, 0), (0x80, 64)])
def test_constant_extremes(byte, re):
    # closed form T*(a^2 + b^2): 0x00 = (-8,-8) -> 128, 0xFF = (7,7) -> 98, 0x80 = (0,-8) -> 64
    t = 1000
    x = synth.constant_bytes(3, t, 200, byte, device=DEV)
    vis = gpu_correlate(x).cpu().numpy()
    assert (vis[..., 0] == re * t).all() and (vis[..., 1] == 0).all()


def test_accumulate_frames_equals_one_long_frame():
    x = synth.quantized_gaussian(2, 600, 150, 2.5, seed=9)
    xd = x.to(DEV)
    whole = gpu_correlate(xd)
    first = gpu_correlate(xd[:, :250].contiguous())
    both = gpu_correlate(xd[:, 250:].contiguous(), prev=first, t_prev=250)
    assert torch.equal(whole, both)
    assert_same(both, oracle.correlate(x.numpy()))


@pytest.mark.parametrize("split", [2, 3, 7, 64])
def test_time_split_bit_identical(split):
    x = synth.quantized_gaussian(2, 1000, 300, 2.5, seed=split)
    xd = x.to(DEV)
    ref = gpu_correlate(xd, variant=0, split=1)
    got = gpu_correlate(xd, variant=0, split=split)
    assert torch.equal(ref, got)
    prev = torch.randint(-1000, 1000, ref.shape, dtype=torch.int32, device=DEV)
    got2 = gpu_correlate(xd, variant=0, split=split, prev=prev.clone(), t_prev=10)
    assert torch.equal(got2, ref + prev)


def test_repeat_runs_bit_identical():
    x = synth.uniform_bytes(4, 512, 384, seed=5, device=DEV)
    a = gpu_correlate(x)
    b = gpu_correlate(x)
    assert torch.equal(a, b)


def test_unaligned_input_pointer():
    # input starting one byte into an allocation: the byte-load path
    x = synth.uniform_bytes(1, 1 * 130 * 64 + 1, 1, seed=3).reshape(-1)
    body = x[1:].reshape(1, 130, 64)
    xd = torch.empty(x.numel(), dtype=torch.uint8, device=DEV)
    xd.copy_(x.to(DEV))
    view = xd[1:].view(1, 130, 64)
    assert view.data_ptr() % 4 == 1
    vis = gpu_correlate(view)
    assert_same(vis, oracle.correlate(body.numpy()))


def test_pathfinder_full_size():
    # N=256, F=256, T=16384, sigma 2.5 with a 0.3 common component
    w = workloads.PATHFINDER
    xd = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seed, common=w.common, device=DEV)
    vis = gpu_correlate(xd)
    x = xd.cpu().numpy()
    for ch in (0, w.f - 1):
        assert_same(vis[ch:ch + 1], oracle.correlate(x[ch:ch + 1]), "channel %d" % ch)
    elems = boundary_elements(w.n, extra=16)
    assert_same(gather_subset(vis, w.n, elems), subset_reference(x, elems), "subset")


def test_large_n_four_frames_accumulated():
    # N=2048, F=16, T=65536 per frame, sigma 3, 4 frames summed on the device
    w = workloads.LARGE_N
    elems = boundary_elements(w.n, extra=8, offsets=(-1, 0))
    vis = None
    want = None
    for k, seed in enumerate(w.seeds()):
        xd = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, seed, device=DEV)
        vis = gpu_correlate(xd, prev=vis, t_prev=k * w.t)
        sub = xd[:, :, torch.as_tensor(elems, device=DEV)].cpu().numpy()
        part = oracle.correlate(sub)
        want = part if want is None else want + part
        del xd
    assert_same(gather_subset(vis, w.n, elems), want, "large-N subset")


VARIANT_SHAPES = [(1, 64, 4), (2, 97, 128), (1, 200, 256), (2, 333, 260), (1, 1000, 384),
                  (1, 130, 512), (3, 64, 132), (1, 4097, 256), (2, 1, 1024)]


TRI_VARIANT = 3
TRI_BF6_VARIANT = 4
TRI_VARIANTS = [TRI_VARIANT, TRI_BF6_VARIANT]
RECT_VARIANT = 5
SMALL_VARIANT = 6
RECT_BF6_VARIANT = 7
RECT_VARIANTS = [RECT_VARIANT, RECT_BF6_VARIANT]


@pytest.mark.parametrize("variant", [0, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("f,t,n", VARIANT_SHAPES)
def test_each_variant_matches_oracle(variant, f, t, n):
    x = synth.quantized_gaussian(f, t, n, 3.0, seed=f * 7919 + t * 31 + n)
    if (variant in TRI_VARIANTS and n > 256) or (variant == SMALL_VARIANT and n > 64):
        import paper_1503_06203_amd as xe
        with pytest.raises(xe.XengError):
            gpu_correlate(x.to(DEV), variant=variant, split=1)
        return
    full_check(x, variant=variant, split=1)


# Triangle kernel (n <= 256, one workgroup per channel): element counts over
# every 32-block edge, and sample counts around the 64-sample stage edges
# where the steady loop hands over to the drain (1, 2 and 3 stages left).
@pytest.mark.parametrize("n", [4, 8, 32, 36, 60, 64, 96, 124, 128, 132, 160, 192, 220, 224, 228,
                               252, 256])
@pytest.mark.parametrize("tv", TRI_VARIANTS)
def test_tri_element_counts(n, tv):
    x = synth.quantized_gaussian(2, 301, n, 3.0, seed=1000 + n)
    full_check(x, variant=tv, split=1)


@pytest.mark.parametrize("t", [1, 7, 8, 9, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256,
                               257, 319, 320, 321, 448, 1000])
@pytest.mark.parametrize("tv", TRI_VARIANTS)
def test_tri_sample_counts(t, tv):
    x = synth.quantized_gaussian(1, t, 256, 2.5, seed=2000 + t)
    full_check(x, variant=tv, split=1)


@pytest.mark.parametrize("split", [2, 3, 5, 16])
@pytest.mark.parametrize("t", [200, 1000, 4097])
@pytest.mark.parametrize("tv", TRI_VARIANTS)
def test_tri_time_split(split, t, tv):
    x = synth.quantized_gaussian(3, t, 192, 2.5, seed=split * 31 + t)
    xd = x.to(DEV)
    ref = gpu_correlate(xd, variant=0, split=1)
    got = gpu_correlate(xd, variant=tv, split=split)
    assert torch.equal(ref, got)
    assert_same(got, oracle.correlate(x.numpy()))
    prev = torch.randint(-1000, 1000, ref.shape, dtype=torch.int32, device=DEV)
    got2 = gpu_correlate(xd, variant=tv, split=split, prev=prev.clone(), t_prev=10)
    assert torch.equal(got2, ref + prev)


@pytest.mark.parametrize("tv", TRI_VARIANTS)
def test_tri_accumulate_and_many_channels(tv):
    x = synth.quantized_gaussian(300, 130, 100, 2.5, seed=61)
    xd = x.to(DEV)
    first = gpu_correlate(xd[:, :70].contiguous(), variant=tv)
    both = gpu_correlate(xd[:, 70:].contiguous(), variant=tv, prev=first, t_prev=70)
    assert_same(both, oracle.correlate(x.numpy()))


@pytest.mark.parametrize("tv", TRI_VARIANTS)
def test_tri_offset_sums_wrap_exactly(tv):
    # The triangle kernel multiplies the 4-bit fields (0..15) and subtracts
    # field sums afterwards. With every byte 0xFF over the longest allowed
    # integration in one workgroup, the uncorrected sums (450 per sample) wrap
    # int32 three times; the corrected result, 98 per sample, does not.
    import paper_1503_06203_amd as xe
    t = xe.MAX_SAMPLES
    x = synth.constant_bytes(1, t, 8, 0xFF, device=DEV)
    vis = gpu_correlate(x, variant=tv, split=1).cpu().numpy()
    assert (vis[..., 0] == 98 * t).all() and (vis[..., 1] == 0).all()


@pytest.mark.parametrize("tv", TRI_VARIANTS)
def test_tri_constant_extremes_exercise_masking(tv):
    # 0x00 decodes to (-8,-8); any padded sample read as 0x00 instead of a
    # zero sample would add 128 per entry
    for t in (1, 65, 200):
        x = synth.constant_bytes(2, t, 256, 0x00, device=DEV)
        vis = gpu_correlate(x, variant=tv).cpu().numpy()
        assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all()


@pytest.mark.parametrize("t", [131008, 131072, 262144 + 64])
def test_tri_bf6_fp32_range(t):
    # every byte 0x00 is (-8, -8): Re grows by 128 per sample, the most any
    # sample adds. A bf6 part sums at most 131 008 samples (fp32 exact below
    # 2^24); longer runs must be split whatever split the caller asks for.
    x = synth.constant_bytes(1, t, 64, 0x00, device=DEV)
    vis = gpu_correlate(x, variant=TRI_BF6_VARIANT, split=1).cpu().numpy()
    assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all()


def test_long_integration_windows():
    # T above 2^20 samples: parts of the time axis that each stay far below
    # the int32 range of one workgroup's sums
    x = synth.quantized_gaussian(1, 1_100_000, 64, 2.5, seed=77)
    full_check(x)


def test_int32_boundary_on_gpu():
    # T = 16 777 215 samples of (-8,-8): Re = 128*T = 2 147 483 520, the int32 limit
    import paper_1503_06203_amd as xe
    t = xe.MAX_SAMPLES
    x = torch.zeros((1, t, 8), dtype=torch.uint8, device=DEV)
    vis = gpu_correlate(x).cpu().numpy()
    assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all()
    v2 = xe.new_vis(8, 1, device=DEV)
    with pytest.raises(xe.XengError):
        xe.correlate(x[:, :1].contiguous(), v2, t_prev=t, accumulate=True)


# Diagonal squares and off-diagonal tiles (n > 256): element counts around the
# 128-row and 256-column edges, with partial last squares and tiles.
@pytest.mark.parametrize("n", [260, 264, 380, 384, 388, 508, 512, 516, 636, 640, 768, 772, 1020,
                               1024, 1028])
@pytest.mark.parametrize("rv", RECT_VARIANTS)
def test_rect_element_counts(n, rv):
    x = synth.quantized_gaussian(2, 301, n, 3.0, seed=3000 + n)
    full_check(x, variant=rv, split=1)


@pytest.mark.parametrize("t", [1, 7, 63, 64, 65, 127, 128, 129, 191, 192, 193, 257, 1000])
@pytest.mark.parametrize("rv", RECT_VARIANTS)
def test_rect_sample_counts(t, rv):
    x = synth.quantized_gaussian(1, t, 512, 2.5, seed=4000 + t)
    full_check(x, variant=rv, split=1)


@pytest.mark.parametrize("split", [2, 3, 5, 16])
@pytest.mark.parametrize("t", [200, 1000, 4097])
@pytest.mark.parametrize("rv", RECT_VARIANTS)
def test_rect_time_split(split, t, rv):
    x = synth.quantized_gaussian(2, t, 516, 2.5, seed=split * 37 + t)
    xd = x.to(DEV)
    ref = gpu_correlate(xd, variant=0, split=1)
    got = gpu_correlate(xd, variant=rv, split=split)
    assert torch.equal(ref, got)
    assert_same(got, oracle.correlate(x.numpy()))
    prev = torch.randint(-1000, 1000, ref.shape, dtype=torch.int32, device=DEV)
    got2 = gpu_correlate(xd, variant=rv, split=split, prev=prev.clone(), t_prev=10)
    assert torch.equal(got2, ref + prev)


@pytest.mark.parametrize("rv", RECT_VARIANTS)
def test_rect_accumulate_and_many_channels(rv):
    x = synth.quantized_gaussian(40, 130, 300, 2.5, seed=71)
    xd = x.to(DEV)
    first = gpu_correlate(xd[:, :70].contiguous(), variant=rv)
    both = gpu_correlate(xd[:, 70:].contiguous(), variant=rv, prev=first, t_prev=70)
    assert_same(both, oracle.correlate(x.numpy()))


@pytest.mark.parametrize("t", [131008, 131072, 262208])
def test_rect_bf6_fp32_range(t):
    # 0x00 bytes decode to (-8, -8): every sample adds 128 to Re of every pair.
    # One workgroup may sum at most 131 008 samples in fp32 (2047 stages);
    # beyond, the library raises the time split. Squares and tiles alike.
    x = synth.constant_bytes(1, t, 520, 0x00, device=DEV)
    vis = gpu_correlate(x, variant=RECT_BF6_VARIANT, split=1).cpu().numpy()
    assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all()


def test_rect_bf6_equals_int8_on_large_n_frame():
    # the full-CHIME array size: bf6 and int8 give the same integers, and one
    # whole channel matches the oracle
    x = synth.quantized_gaussian(2, 8192, 2048, 3.0, seed=77)
    xd = x.to(DEV)
    a = gpu_correlate(xd, variant=RECT_BF6_VARIANT)
    b = gpu_correlate(xd, variant=RECT_VARIANT)
    assert torch.equal(a, b)
    assert_same(a[:1], oracle.correlate(x[:1].numpy()), "bf6 channel 0")


def test_rect_offset_sums_wrap_exactly():
    # every byte 0xFF over the longest allowed integration in one workgroup:
    # the uncorrected field products of a square and of a tile wrap int32, the
    # corrected result (98 per sample) does not
    import paper_1503_06203_amd as xe
    t = xe.MAX_SAMPLES
    x = synth.constant_bytes(1, t, 264, 0xFF, device=DEV)
    vis = gpu_correlate(x, variant=RECT_VARIANT, split=1).cpu().numpy()
    assert (vis[..., 0] == 98 * t).all() and (vis[..., 1] == 0).all()


def test_rect_constant_extremes_exercise_masking():
    # 0x00 decodes to (-8,-8): a padded sample or element read as 0x00 instead
    # of a zero field would add 128 per entry
    for t in (1, 65, 200):
        x = synth.constant_bytes(2, t, 520, 0x00, device=DEV)
        vis = gpu_correlate(x, variant=RECT_VARIANT).cpu().numpy()
        assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all()


def test_large_n_one_channel_in_full():
    # one channel of a large-N frame (N=2048, T=65536, sigma 3), every entry
    # against the oracle: 1.4e11 complex multiply-adds on the host
    w = workloads.LARGE_N
    xd = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seeds()[0], device=DEV)
    vis = gpu_correlate(xd)
    ch = w.f - 1
    x = xd[ch:ch + 1].cpu().numpy()
    del xd
    assert_same(vis[ch:ch + 1], oracle.correlate(x), "channel %d" % ch)


# Small kernel (n <= 64): element counts over the 32-block edge, sample counts
# around the 16-sample steps and the time parts, channel counts around the
# packing of channels into workgroups (all parts of a channel in one).
@pytest.mark.parametrize("n", [4, 8, 12, 28, 32, 36, 60, 64])
@pytest.mark.parametrize("t", [1, 15, 16, 17, 255, 257, 4097])
def test_small_element_and_sample_counts(n, t):
    x = synth.quantized_gaussian(2, t, n, 3.0, seed=5000 + 97 * n + t)
    full_check(x, variant=SMALL_VARIANT)


@pytest.mark.parametrize("f", [1, 3, 255, 256, 257, 700, 1025])
def test_small_channel_counts(f):
    x = synth.quantized_gaussian(f, 200, 64, 2.5, seed=6000 + f)
    full_check(x, variant=SMALL_VARIANT)


def test_small_accumulate():
    x = synth.quantized_gaussian(5, 3000, 48, 2.5, seed=81)
    xd = x.to(DEV)
    first = gpu_correlate(xd[:, :1300].contiguous(), variant=SMALL_VARIANT)
    both = gpu_correlate(xd[:, 1300:].contiguous(), variant=SMALL_VARIANT, prev=first,
                         t_prev=1300)
    assert_same(both, oracle.correlate(x.numpy()))


def test_small_offset_sums_wrap_exactly():
    # one channel split over the 8 waves of a workgroup: each part's
    # uncorrected field products wrap int32; the parts combine modulo 2^32
    import paper_1503_06203_amd as xe
    t = xe.MAX_SAMPLES
    x = synth.constant_bytes(1, t, 64, 0xFF, device=DEV)
    vis = gpu_correlate(x, variant=SMALL_VARIANT).cpu().numpy()
    assert (vis[..., 0] == 98 * t).all() and (vis[..., 1] == 0).all()


def test_small_constant_extremes_exercise_masking():
    for n in (60, 64, 20):
        for t in (1, 17, 200):
            x = synth.constant_bytes(3, t, n, 0x00, device=DEV)
            vis = gpu_correlate(x, variant=SMALL_VARIANT).cpu().numpy()
            assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all(), (n, t)


def test_small_n_workload_full_size():
    # N=64, F=1024, T=16384: every channel's entries against the oracle on a
    # channel sample, plus all channels of a 3-element subset
    w = workloads.SMALL_N
    xd = synth.quantized_gaussian(w.f, w.t, w.n, w.sigma, w.seed, device=DEV)
    vis = gpu_correlate(xd)
    for ch in (0, 511, w.f - 1):
        assert_same(vis[ch:ch + 1], oracle.correlate(xd[ch:ch + 1].cpu().numpy()), "ch %d" % ch)
    elems = np.array([0, 31, 63])
    sub = xd[:, :, torch.as_tensor(elems, device=DEV)].cpu().numpy()
    assert_same(gather_subset(vis, w.n, elems), oracle.correlate(sub), "subset")
