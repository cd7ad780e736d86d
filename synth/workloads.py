"""The named workloads: shapes, value distributions and seeds.

All inputs are synthetic (see ``synth`` for the sample recipe). The sizes are
those of the instruments the paper targets: the CHIME Pathfinder (N = 256
elements) and full CHIME (N = 2048), plus batched and streamed mixes of jobs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    f: int
    t: int
    sigma: float
    seed: int
    common: float = 0.0
    frames: int = 1
    frame_seeds: tuple = field(default_factory=tuple)

    def seeds(self):
        return self.frame_seeds if self.frame_seeds else (self.seed,)

    @property
    def effective_ops_per_frame(self) -> int:
        # Eq. 2: 8 operations per upper-triangle entry per channel per sample
        return 8 * (self.n * (self.n + 1) // 2) * self.f * self.t


TINY = Workload("tiny", n=16, f=1, t=256, sigma=2.5, seed=1)
PATHFINDER = Workload("pathfinder", n=256, f=256, t=16384, sigma=2.5, seed=2, common=0.3)
LARGE_N = Workload("large_n", n=2048, f=16, t=65536, sigma=3.0, seed=30, frames=4,
                   frame_seeds=(30, 31, 32, 33))

# Small arrays are bound by HBM, not by the matrix cores: at N = 64 one input
# byte carries 4 (N + 1) = 260 effective operations, under the ~625 op/B ridge
# of the int8 MFMA peak against 8 TB/s. 1024 channels of 16384 samples are
# 1 GiB of input per frame.
SMALL_N = Workload("small_n", n=64, f=1024, t=16384, sigma=2.5, seed=6)

WORKLOADS = {w.name: w for w in (TINY, PATHFINDER, LARGE_N, SMALL_N)}


def batched_jobs(seed: int = 4, count: int = 64):
    """64 correlation jobs of mixed size for the one-launch batched mode.

    N from {64, 256, 512, 1024, 2048}, F uniform in [1, 32], T uniform in
    [4096, 65536] (most T are not a multiple of any tile depth, which exercises
    the ragged tails), sigma 2.5. Returns a list of dicts with a per-job seed.
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array([64, 256, 512, 1024, 2048]), size=count)
    fs = rng.integers(1, 33, size=count)
    ts = rng.integers(4096, 65537, size=count)
    return [dict(n=int(n), f=int(f), t=int(t), sigma=2.5, seed=1000 * seed + k)
            for k, (n, f, t) in enumerate(zip(ns, fs, ts))]


def served_stream(seed: int = 5, rate_hz: float = 2000.0, frames: int = 400,
                  n_choices=(256, 2048, 8192), n_weights=(0.6, 0.35, 0.05),
                  f_choices=(1, 2, 8), t: int = 16384):
    """Poisson arrivals of correlation frames for the serving mode.

    Inter-arrival times are exponential with mean 1/rate_hz. Each frame belongs
    to a job; a job is one (N, F) stream whose accumulator lives on the device.
    N is drawn with ``n_weights`` and F uniformly from ``f_choices``.
    Returns (arrival_s, n, f) arrays.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=frames)
    arrivals = np.cumsum(gaps) - gaps[0]
    p = np.asarray(n_weights, dtype=np.float64)
    n = rng.choice(np.asarray(n_choices), size=frames, p=p / p.sum())
    f = rng.choice(np.asarray(f_choices), size=frames)
    return arrivals, n.astype(np.int64), f.astype(np.int64), t
