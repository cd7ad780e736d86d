"""Strided inputs: the time-major packet stream [T][F][N] of Sec. III (Fig. 2)
and padded sample rows, read in place. The expected values come from the
oracle on a dense [F][T][N] copy made on the host (a pure re-indexing)."""
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


def correlate_view(xv, prev=None, t_prev=0):
    import paper_1503_06203_amd as xe
    f, t, n = xv.shape
    vis = xe.new_vis(n, f, device=DEV)
    if prev is not None:
        vis.copy_(prev)
    xe.correlate(xv, vis, t_prev=t_prev, accumulate=prev is not None)
    torch.cuda.synchronize()
    return vis


@pytest.mark.parametrize("f,t,n", [(4, 1000, 256), (3, 97, 64), (2, 700, 384), (5, 130, 132),
                                   (2, 4097, 1024), (2, 65, 4)])
def test_time_major_stream_matches_oracle(f, t, n):
    dense = synth.quantized_gaussian(f, t, n, 2.5, seed=f * 131 + t + n)
    stream = dense.permute(1, 0, 2).contiguous()            # [T][F][N] in memory
    view = stream.to(DEV).permute(1, 0, 2)                  # [F][T][N] view, strides (n, f*n, 1)
    assert not view.is_contiguous() and view.stride(1) == f * n and view.stride(0) == n
    assert_same(correlate_view(view), oracle.correlate(dense.numpy()), "time-major")


@pytest.mark.parametrize("n,pad", [(256, 4), (200, 56), (512, 32)])
def test_padded_sample_rows(n, pad):
    f, t = 3, 333
    full = synth.uniform_bytes(f, t, n + pad, seed=n + pad)
    view = full.to(DEV)[:, :, :n]                           # sample stride n + pad
    assert view.stride(1) == n + pad
    assert_same(correlate_view(view), oracle.correlate(np.ascontiguousarray(full.numpy()[:, :, :n])),
                "padded rows")


def test_time_major_equals_dense_at_scale_and_accumulates():
    f, t, n = 32, 4096, 256
    dense = synth.quantized_gaussian(f, t, n, 2.5, seed=77, common=0.3, device=DEV)
    view = dense.permute(1, 0, 2).contiguous().permute(1, 0, 2)
    a = correlate_view(dense)
    b = correlate_view(view)
    assert torch.equal(a, b)
    c = correlate_view(view, prev=a, t_prev=t)
    assert torch.equal(c, a + a)
    x = dense.cpu().numpy()
    assert_same(b[:2], oracle.correlate(x[:2]), "two channels")


def test_strided_layout_errors():
    import paper_1503_06203_amd as xe
    full = torch.zeros((2, 10, 66), dtype=torch.uint8, device=DEV)
    vis = xe.new_vis(64, 2, device=DEV)
    with pytest.raises(xe.XengError):                         # sample stride 66: not a multiple of 4
        xe.correlate(full[:, :, :64], vis)
    with pytest.raises(TypeError):                            # elements not contiguous
        xe.correlate(torch.zeros((2, 64, 10), dtype=torch.uint8, device=DEV).transpose(1, 2), vis)
