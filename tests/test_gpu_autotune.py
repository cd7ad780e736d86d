"""The autotuner of plain calls: it times every variant that can run a job,
keeps the fastest for the job's class, and later calls of that class use it;
results stay the oracle's integers whichever variant runs."""
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


@pytest.mark.parametrize("n,f,t", [(260, 2, 3000), (64, 3, 700), (128, 1, 1100)])
def test_autotune_records_reloads_and_stays_exact(n, f, t, tmp_path):
    print("autotune n=%d f=%d t=%d" % (n, f, t), flush=True)
    xe.tune_clear()
    cache = tmp_path / "tune.txt"
    x = synth.quantized_gaussian(f, t, n, 2.5, seed=n + t)
    vis = xe.new_vis(n, f)
    vis.fill_(-5)
    v, split, ms = xe.autotune(x.to(DEV), vis, reps=2, tune_cache=cache)
    torch.cuda.synchronize()
    assert 0 <= v < len(xe.variants()) and ms > 0
    assert np.array_equal(vis.cpu().numpy().astype(np.int64), oracle.correlate(x.numpy()))
    line = cache.read_text().split()
    assert line[0] == "xeng-tune" and line[2:7] == [str(n), str(f), str(t.bit_length() - 1),
                                                    str(v), str(split)]
    assert xe.choose_variant(n, f, t)[0] == v
    # another frame of the same class (t within the same power of two) runs
    # the tuned variant and gives the oracle's sums
    t2 = t - 37
    x2 = synth.quantized_gaussian(f, t2, n, 2.5, seed=n + t2 + 1)
    assert xe.choose_variant(n, f, t2)[0] == v
    got = xe.correlate(x2.to(DEV), xe.new_vis(n, f))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.int64), oracle.correlate(x2.numpy()))
    # forgotten, then reloaded from the cache file
    xe.tune_clear()
    assert xe.tune_load(cache) == 1
    assert xe.choose_variant(n, f, t2)[0] == v
    xe.tune_clear()
