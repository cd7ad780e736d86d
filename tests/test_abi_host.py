"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and its index helpers and argument checks behave as
documented. No call here reaches the GPU: every correlate call below is
rejected by the argument checks before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xengine.h")

EINVAL, ERANGE, ENOTFOUND = -1, -2, -6
FAKE_IN = 0x10000000
FAKE_VIS = 0x20000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xeng_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1503_06203_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(lib):
    from paper_1503_06203_amd import _lib
    names = declared_functions()
    assert "xeng_correlate" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, "binding lacks " + name


def test_tri_index_is_row_major_bijection(lib):
    for n in (1, 2, 3, 7, 64, 129):
        i, j = np.triu_indices(n)
        ks = [lib.xeng_tri_index(n, int(a), int(b)) for a, b in zip(i, j)]
        assert ks == list(range(n * (n + 1) // 2))
        assert lib.xeng_vis_entries(n) == n * (n + 1) // 2
    assert lib.xeng_tri_index(4, 2, 1) == -1
    assert lib.xeng_tri_index(4, 0, 4) == -1
    assert lib.xeng_tri_index(4, -1, 0) == -1
    big = 46341  # entries exceed 2^31
    assert lib.xeng_tri_index(big, big - 1, big - 1) == big * (big + 1) // 2 - 1


def test_tile_count_fig1(lib):
    assert lib.xeng_tile_count(256, 32) == 36      # Fig. 1
    assert lib.xeng_tile_count(2048, 128) == 136
    assert lib.xeng_tile_count(257, 128) == 6
    assert lib.xeng_tile_count(0, 32) == -1


def call(lib, n=16, f=1, t=8, t_prev=0, acc=0, d_in=FAKE_IN, d_vis=FAKE_VIS, variant=0, split=1):
    return lib.xeng_correlate_variant(d_in, d_vis, n, f, t, t_prev, acc, variant, split, None)


def test_rejects_bad_shapes(lib):
    assert call(lib, n=0) == EINVAL
    assert call(lib, f=0) == EINVAL
    assert call(lib, t=-1) == EINVAL
    assert "n >= 1" in lib.xeng_last_error().decode()
    assert call(lib, acc=2) == EINVAL
    assert call(lib, d_vis=None) == EINVAL
    assert call(lib, d_in=None) == EINVAL
    assert call(lib, d_vis=FAKE_VIS + 4) == EINVAL        # not 8-byte aligned
    assert call(lib, split=-1) == EINVAL


def test_rejects_overlap(lib):
    # input [1][8][16] = 128 bytes; output starts inside it
    assert call(lib, d_vis=FAKE_IN + 64) == EINVAL
    assert "overlap" in lib.xeng_last_error().decode()


def test_range_guard(lib):
    m = 16_777_215
    assert call(lib, t=8, t_prev=m - 7, acc=1) == ERANGE
    assert call(lib, t=8, t_prev=5, acc=0) == EINVAL      # t_prev only when accumulating
    assert call(lib, t=8, t_prev=-1, acc=1) == EINVAL


def test_unknown_variant(lib):
    assert call(lib, variant=lib.xeng_variant_count()) == ENOTFOUND
    # the retired 128 x 256 wide kernels are refused (variant 5 covers them)
    assert call(lib, variant=1) == ENOTFOUND and call(lib, variant=2) == ENOTFOUND
    assert lib.xeng_variant_name(1).startswith(b"retired")
    assert lib.xeng_variant_name(-5) is None
    assert lib.xeng_variant_name(0) is not None


def test_choose_variant_dispatch_rule():
    # small kernel for aligned n <= 64, triangle kernel for aligned n <= 256
    # with n % 4 == 0; diagonal squares and
    # off-diagonal tiles for other aligned n % 4 == 0; the general kernel otherwise
    import paper_1503_06203_amd as xe
    assert xe.choose_variant(256, 256, 16384)[2].startswith("tri256")
    assert xe.choose_variant(68, 1, 10)[2].startswith("tri256")
    # arrays of at most 64 elements stream through the small kernel
    assert xe.choose_variant(4, 1, 10)[2].startswith("small64")
    assert xe.choose_variant(64, 1024, 16384)[2].startswith("small64")
    assert xe.choose_variant(260, 4, 100)[2].startswith("rect128x256")
    assert xe.choose_variant(2048, 16, 65536)[2].startswith("rect128x256")
    # the large-N frame (16 channels x 64 pieces) fills 4 whole rounds of the
    # 256 compute units without splitting the time axis
    assert xe.choose_variant(2048, 16, 65536)[1] == 1
    assert xe.choose_variant(255, 4, 100)[2].startswith("tile128")
    assert xe.choose_variant(256, 4, 100, aligned=False)[2].startswith("tile128")
    # one channel of a long integration is split in time across workgroups
    v, split, _ = xe.choose_variant(256, 1, 1 << 20)
    assert split > 1
    assert xe.choose_variant(256, 256, 16384)[1] == 1
    with pytest.raises(xe.XengError):
        xe.choose_variant(0, 1, 1)


def test_strided_validation(lib):
    st = lib.xeng_correlate_strided
    # sample stride below n, or not a multiple of 4, or an unaligned base
    assert st(FAKE_IN, 60, 64 * 10, FAKE_VIS, 64, 2, 10, 0, 0, None) == EINVAL
    assert st(FAKE_IN, 66, 66 * 10, FAKE_VIS, 64, 2, 10, 0, 0, None) == EINVAL
    assert st(FAKE_IN + 2, 128, 1280, FAKE_VIS, 64, 2, 10, 0, 0, None) == EINVAL
    # a sample stride whose 32-bit buffer offsets would overflow
    assert st(FAKE_IN, 1 << 27, 64, FAKE_VIS, 64, 2, 10, 0, 0, None) == EINVAL
    # the strided extent reaches the output: time-major [T][F][N], vis right after
    n, f, t = 64, 4, 100
    assert st(FAKE_IN, f * n, n, FAKE_IN + t * f * n - 64, n, f, t, 0, 0, None) == EINVAL
    assert b"overlap" in lib.xeng_last_error()


def test_python_binding_errors_without_gpu():
    import torch
    import paper_1503_06203_amd as xe
    x = torch.zeros((1, 4, 4), dtype=torch.uint8)
    v = torch.zeros((1, 10, 2), dtype=torch.int32)
    with pytest.raises(TypeError):
        xe.correlate(x, v)            # CPU tensors: there is no CPU path


def test_plan_host_logic(lib):
    """Plan building is host-only: item counts, workspace size, validation."""
    from paper_1503_06203_amd._lib import XengJob
    import ctypes
    jobs = (XengJob * 3)()
    base_in, base_vis = 0x100000000, 0x900000000
    shapes = [(256, 2, 1000), (64, 1, 64), (2048, 1, 100)]
    for k, (n, f, t) in enumerate(shapes):
        jobs[k] = XengJob(base_in + k * (1 << 28), base_vis + k * (1 << 28), n, f, t, 0, 0)
    h = ctypes.c_void_p()
    assert lib.xeng_plan_create(ctypes.byref(h), jobs, 3, None) == 0
    # N <= 256 is one diagonal square (the whole triangle) per channel (2 + 1);
    # N=2048 is 8 squares plus the 56 128x256 tiles above them per channel
    assert lib.xeng_plan_items(h) == 2 + 1 + 64
    assert lib.xeng_plan_split(h) == 1
    assert lib.xeng_plan_workspace_bytes(h) > 0
    lib.xeng_plan_destroy(h)
    jobs[1] = XengJob(base_in, base_vis, 6, 1, 10, 0, 0)        # n % 4 != 0
    assert lib.xeng_plan_create(ctypes.byref(h), jobs, 3, None) == EINVAL
    assert b"n % 4" in lib.xeng_last_error()


def test_static_plan_run_refuses_oversize_plan(lib):
    """xeng_plan_run_static refuses, before any device work, a plan whose image
    exceeds the static device array: 4097 channels x 64 pieces at N=2048 is
    262 208 queue items of 32 bytes, more than XENG_STATIC_SCRATCH_BYTES."""
    from paper_1503_06203_amd._lib import XengJob
    import ctypes
    text = open(HEADER).read()
    limit = int(re.search(r"XENG_STATIC_SCRATCH_BYTES \((\d+)LL << (\d+)\)", text).group(1)) << 20
    assert limit == 8 << 20
    jobs = (XengJob * 1)()
    jobs[0] = XengJob(0x100000000, 0x10000000000, 2048, 4097, 64, 0, 0)
    h = ctypes.c_void_p()
    assert lib.xeng_plan_create(ctypes.byref(h), jobs, 1, None) == 0
    assert lib.xeng_plan_items(h) == 4097 * 64
    assert lib.xeng_plan_run_static(h, None) == EINVAL
    assert b"static scratch" in lib.xeng_last_error()
    lib.xeng_plan_destroy(h)
    assert lib.xeng_plan_run_static(None, None) == EINVAL


def test_tune_table_host(lib, tmp_path):
    """The autotuner's table and cache file on the host: without a device the
    architecture reads "none", so lines for "none" apply and others do not;
    a tuned (variant, split) replaces the default choice for its class
    (n, f, floor(log2 t)) only, where the variant can run the job."""
    import paper_1503_06203_amd as xe
    xe.tune_clear()
    default = xe.choose_variant(300, 2, 3000)
    assert default[2].startswith("rect128x256")
    default_t5000 = xe.choose_variant(300, 2, 5000)
    default_f3 = xe.choose_variant(300, 3, 3000)
    cache = tmp_path / "tune.txt"
    cache.write_text("xeng-tune none 300 2 11 7 4 1.5\n"      # rect bf6, split 4, t in [2048, 4096)
                     "xeng-tune gfx000 300 2 11 0 1 1.0\n"    # another device: skipped
                     "garbage line\n"
                     "xeng-tune none 300 2 11 0 2 1.2\n"      # a later line replaces the first
                     "xeng-tune none 64 1 8 3 0 0.1\n"        # tri256 with its own split
                     "xeng-tune none 512 2 11 1 1 0.9\n")     # a retired variant: never used
    assert xe.tune_load(cache) == 4
    v, split, name = xe.choose_variant(300, 2, 3000)
    assert (v, split) == (0, 2) and name.startswith("tile128")
    assert xe.choose_variant(512, 2, 3000)[2].startswith("rect128x256")
    assert xe.choose_variant(300, 2, 5000) == default_t5000            # other t bucket
    assert xe.choose_variant(300, 3, 3000) == default_f3               # other f
    # a tuned variant that cannot run the call (unaligned input) is not used
    assert xe.choose_variant(300, 2, 3000, aligned=False)[2].startswith("tile128")
    assert xe.choose_variant(64, 1, 300)[2].startswith("tri256")
    xe.tune_clear()
    assert xe.choose_variant(300, 2, 3000)[:2] == default[:2]
    assert xe.choose_variant(64, 1, 300)[2].startswith("small64")
    with pytest.raises(xe.XengError) as e:
        xe.tune_load(tmp_path / "missing.txt")
    assert e.value.status == ENOTFOUND
