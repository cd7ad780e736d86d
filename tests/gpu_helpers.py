"""Shared pieces of the GPU tests: run the HIP path, fetch results, compare
with the oracle element by element (tolerance 0: all arithmetic is integer)."""
import numpy as np
import torch

import oracle
import paper_1503_06203_amd as xe
import synth


def gpu_correlate(x_dev, variant=None, split=1, prev=None, t_prev=0):
    f, t, n = x_dev.shape
    vis = xe.new_vis(n, f, device=x_dev.device)
    acc = prev is not None
    if acc:
        vis.copy_(prev)
    if variant is None:
        xe.correlate(x_dev, vis, t_prev=t_prev, accumulate=acc)
    else:
        xe.correlate_variant(x_dev, vis, variant, split, t_prev=t_prev, accumulate=acc)
    torch.cuda.synchronize()
    return vis


def assert_same(got_i32, want_i64, what=""):
    got = got_i32.cpu().numpy().astype(np.int64) if torch.is_tensor(got_i32) else got_i32
    want = np.asarray(want_i64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    if len(bad):
        k = tuple(bad[0])
        raise AssertionError("%s: %d mismatches, first at %s: got %d want %d"
                             % (what, len(bad), k, got[k], want[k]))


def subset_reference(x_cpu, elems):
    """Oracle visibilities of the sub-array of elements ``elems`` (sorted): the
    entries (elems[a], elems[b]) of the full matrix, which depend only on those
    two elements' samples."""
    sub = np.ascontiguousarray(x_cpu[:, :, elems])
    return oracle.correlate(sub)


def gather_subset(vis_dev, n, elems):
    """Entries (elems[a], elems[b]), a <= b, of the GPU result, in the oracle's
    packed order for the subset."""
    e = np.asarray(elems)
    a, b = np.triu_indices(len(e))
    i, j = e[a], e[b]
    k = i * (2 * n - i + 1) // 2 + (j - i)
    idx = torch.as_tensor(k, device=vis_dev.device)
    return vis_dev[:, idx, :].cpu().numpy().astype(np.int64)


def boundary_elements(n, tile=128, extra=24, seed=0, offsets=(-2, -1, 0, 1, 31, 32, 63, 64)):
    """Elements around every tile edge plus random ones, sorted and unique."""
    s = {0, n - 1}
    for b in range(0, n, tile):
        for d in offsets:
            if 0 <= b + d < n:
                s.add(b + d)
    rng = np.random.default_rng(seed)
    s.update(int(v) for v in rng.integers(0, n, size=extra))
    return np.array(sorted(s))
