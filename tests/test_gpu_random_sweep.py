"""Seeded random sweep over every entry point against the oracle: shapes,
input alignment, time splits, variants, gate schedules and delay spreads
drawn at random within each entry point's documented limits, with and without
accumulation, and batched plans of a few such jobs. Complements the
hand-picked cases of the other GPU tests."""
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


def _dev_copy(x, off):
    # device copy of x starting `off` bytes into its allocation
    flat = torch.empty(x.numel() + off, dtype=torch.uint8, device=DEV)
    flat[off:].copy_(x.reshape(-1).to(DEV))
    return flat[off:].view(*x.shape)


def _gen(rng, f, t, n, seed):
    if rng.random() < 0.5:
        return synth.quantized_gaussian(f, t, n, float(rng.uniform(0.5, 4.0)), seed=seed)
    return synth.uniform_bytes(f, t, n, seed=seed)


def _plain(rng, seed):
    import paper_1503_06203_amd as xe
    f, t, n = int(rng.integers(1, 5)), int(rng.integers(0, 2500)), int(rng.integers(1, 520))
    off, acc = int(rng.integers(0, 4)), bool(rng.random() < 0.3)
    case = ("plain", f, t, n, off, acc)
    print(case, flush=True)
    x = _gen(rng, f, t, n, seed)
    xd = _dev_copy(x, off)
    vis = xe.new_vis(n, f)
    want = oracle.correlate(x.numpy()) if t else np.zeros((f, xe.vis_entries(n), 2), np.int64)
    if acc:
        xe.correlate(xd, vis)
        xe.correlate(xd, vis, t_prev=t, accumulate=True)
        want = 2 * want
    else:
        vis.fill_(7)                       # overwritten, also where t == 0
        xe.correlate(xd, vis)
    torch.cuda.synchronize()
    assert_same(vis, want, str(case))


def _variant(rng, seed):
    import paper_1503_06203_amd as xe
    live = [k for k, name in enumerate(xe.variants()) if not name.startswith("retired")]
    v = live[int(rng.integers(0, len(live)))]
    if v in (3, 4):                 # triangle kernels: n <= 256
        n = int(rng.integers(1, 257))
    elif v == 6:                    # small-array kernel: n <= 64
        n = int(rng.integers(1, 65))
    else:
        n = int(rng.integers(1, 600))
    if v != 0:
        n = max(4, n - n % 4)
    f, t = int(rng.integers(1, 5)), int(rng.integers(1, 3000))
    split, acc = int(rng.integers(1, 9)), bool(rng.random() < 0.3)
    case = ("variant", v, f, t, n, split, acc)
    print(case, flush=True)
    x = _gen(rng, f, t, n, seed)
    xd = x.to(DEV)
    vis = xe.new_vis(n, f)
    want = oracle.correlate(x.numpy())
    if acc:
        xe.correlate(xd, vis)
        xe.correlate_variant(xd, vis, v, split, t_prev=t, accumulate=True)
        want = 2 * want
    else:
        vis.fill_(-3)
        xe.correlate_variant(xd, vis, v, split)
    torch.cuda.synchronize()
    assert_same(vis, want, str(case))


def _strided(rng, seed):
    import paper_1503_06203_amd as xe
    f, t, n = int(rng.integers(1, 5)), int(rng.integers(1, 2000)), 4 * int(rng.integers(1, 130))
    case = ("time-major", f, t, n)
    print(case, flush=True)
    dense = _gen(rng, f, t, n, seed)
    view = dense.permute(1, 0, 2).contiguous().to(DEV).permute(1, 0, 2)
    vis = xe.new_vis(n, f)
    xe.correlate(view, vis)
    torch.cuda.synchronize()
    assert_same(vis, oracle.correlate(dense.numpy()), str(case))


def _gated(rng, seed):
    import paper_1503_06203_amd as xe
    gates, n, f = int(rng.integers(1, 5)), 4 * int(rng.integers(1, 100)), int(rng.integers(1, 4))
    block = int(rng.choice([64, 100, 128, 1000, int(rng.integers(1, 300))]))
    t = int(rng.integers(1, 3000))
    sched = rng.integers(0, gates + 1, (t + block - 1) // block).astype(np.uint8)
    sched[sched == gates] = 0xFF                              # blocks left out
    case = ("gated", gates, f, t, n, block)
    print(case, flush=True)
    x = _gen(rng, f, t, n, seed)
    vis = torch.full((gates, f, xe.vis_entries(n), 2), 5, dtype=torch.int32, device=DEV)
    xe.correlate_gated(x.to(DEV), vis, sched, block)
    torch.cuda.synchronize()
    assert_same(vis, oracle.correlate_gated(x.numpy(), sched, block, gates), str(case))


def _delayed(rng, seed):
    import paper_1503_06203_amd as xe
    n, f, t = int(rng.integers(1, 257)), int(rng.integers(1, 4)), 64 * int(rng.integers(1, 30))
    spread = int(rng.choice([0, 1, 50, 128, 129, 400]))
    delays = int(rng.integers(0, 50)) + rng.integers(0, spread + 1, n)
    if rng.random() < 0.3:
        delays[:] = delays[0]                                 # one common delay
    off = int(rng.integers(0, 4)) if rng.random() < 0.3 else 0
    case = ("delayed", f, t, n, spread, off)
    print(case, flush=True)
    x = _gen(rng, f, t + int(delays.max()), n, seed)
    vis = xe.new_vis(n, f)
    vis.fill_(9)
    xe.correlate_delayed(_dev_copy(x, off), vis, delays)
    torch.cuda.synchronize()
    assert_same(vis, oracle.correlate_delayed(x.numpy(), delays), str(case))


def _delayed_shift(rng, seed):
    # the shift form: n above 256 or t not whole 64-sample stages; n % 16 == 0
    # half the time (the ring form), a workspace of a few windows a third of
    # the time
    import paper_1503_06203_amd as xe
    n = int(rng.integers(257, 600)) if rng.random() < 0.7 else int(rng.integers(1, 257))
    if rng.random() < 0.5:
        n = max(16, n - n % 16)
    f, t = int(rng.integers(1, 3)), int(rng.integers(1, 1300))
    if n <= 256 and t % 64 == 0:
        t += 1
    spread = int(rng.choice([0, 1, 37, 128, 129, 400]))
    delays = int(rng.integers(0, 30)) + rng.integers(0, spread + 1, n)
    windows = rng.random() < 0.35
    case = ("delayed-shift", f, t, n, spread, windows)
    print(case, flush=True)
    x = _gen(rng, f, t + int(delays.max()), n, seed)
    vis = xe.new_vis(n, f)
    vis.fill_(4)
    ws = None
    if windows:
        ws = torch.empty(f * n * 128 * int(rng.integers(1, 4)) + 3, dtype=torch.uint8, device=DEV)
    xe.correlate_delayed(x.to(DEV), vis, delays, workspace=ws)
    torch.cuda.synchronize()
    assert_same(vis, oracle.correlate_delayed(x.numpy(), delays), str(case))


def _plan(rng, seed):
    # one persistent launch over a few jobs, some accumulating onto held sums
    import paper_1503_06203_amd as xe
    jobs, wants = [], []
    for k in range(int(rng.integers(1, 7))):
        n, f, t = 4 * int(rng.integers(1, 150)), int(rng.integers(1, 4)), int(rng.integers(1, 3000))
        x = _gen(rng, f, t, n, seed + k)
        want = oracle.correlate(x.numpy())
        vis = xe.new_vis(n, f)
        if rng.random() < 0.4:
            prev = rng.integers(-1000, 1000, tuple(vis.shape)).astype(np.int32)
            vis.copy_(torch.from_numpy(prev))
            jobs.append((x.to(DEV), vis, t, True))
            want = want + prev
        else:
            vis.fill_(11)
            jobs.append((x.to(DEV), vis))
        wants.append(want)
    case = ("plan", [tuple(j[0].shape) + (len(j) > 2,) for j in jobs])
    print(case, flush=True)
    plan = xe.Plan(jobs)
    plan.run()
    torch.cuda.synchronize()
    for j, want in zip(jobs, wants):
        assert_same(j[1], want, str(case))


@pytest.mark.parametrize("seed", [101, 202, 303])
def test_random_sweep(seed):
    rng = np.random.default_rng(seed)
    kinds = [_plain, _variant, _strided, _gated, _delayed, _delayed_shift, _plan]
    for _ in range(120):
        kind = kinds[int(rng.choice(7, p=[0.2, 0.2, 0.12, 0.12, 0.14, 0.12, 0.1]))]
        kind(rng, int(rng.integers(1 << 30)))
