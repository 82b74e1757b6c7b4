"""Seeded workload descriptions: uneven batch scales and forced spike lists."""
from __future__ import annotations

import numpy as np

from .conn_table import FULL_SIZE


def batch_scales(n: int, lo: float, hi: float, seed: int):
    """Instance scales drawn uniformly from [lo, hi) (uneven batch)."""
    rng = np.random.Generator(np.random.Philox(seed))
    return rng.uniform(lo, hi, size=n)


def forced_spike_list(count: int, scale: float, seed: int):
    """`count` distinct neuron ids, spread over the populations in proportion to
    their sizes (the delivery microbenchmark's synthetic spike load)."""
    sizes = np.maximum(1, np.floor(np.asarray(FULL_SIZE, dtype=np.float64) * scale + 0.5)).astype(np.int64)
    total = int(sizes.sum())
    rng = np.random.Generator(np.random.Philox(seed))
    count = min(int(count), total)
    return np.sort(rng.choice(total, size=count, replace=False)).astype(np.int32)
