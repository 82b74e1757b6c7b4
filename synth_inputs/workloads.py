"""Seeded workload descriptions: uneven batch scales, forced spike lists and
the stand-in amplitudes of the DC-input workload."""
from __future__ import annotations

import numpy as np

import json
import os

from .conn_table import FULL_SIZE, K_EXT

_RELAXED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "relaxed_start.json")


def relaxed_start():
    """Inputs of the relaxed initial state (init_mode 2) for the stand-in
    network: per-population mean and standard deviation of the membrane
    potential and of the synaptic current in its steady state, as keyword
    arguments of the library's and the oracle's configurations.  The values
    (relaxed_start.json) were measured on the oracle's run of the full-scale
    network; the file names how."""
    r = json.load(open(_RELAXED))
    return dict(init_mode=2, init_u_mean_mv=r["u_mean"], init_u_sd_mv=r["u_sd"],
                init_i_mean_pa=r["i_mean"], init_i_sd_pa=r["i_sd"])


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


def dc_standin_amplitudes(nu_bg_hz: float = 8.0, w_ext_pa: float = 87.8, tau_syn_ms: float = 0.5):
    """Per-population DC input (pA) standing in for the amplitudes the paper's
    DC-driven workload does not give: the mean current the population's
    Poisson background would inject through the exponential synapse,
    K_ext * nu_bg * w_ext * tau_syn (rate times charge per spike)."""
    return tuple(k * nu_bg_hz * w_ext_pa * tau_syn_ms * 1e-3 for k in K_EXT)
