"""Spike-train statistics of Sec. 4b of Rhodes et al. (arXiv 1909.08665):
per-population firing rate, coefficient of variation of the inter-spike
interval, and correlation coefficient of binned spike trains, after discarding
the initial transient (the paper drops the first 1 s, Sec. 2a).

TEST INFRASTRUCTURE ONLY: applied to rasters from the oracle and from the GPU
library alike; neither the simulator nor its kernels use it.
"""
from __future__ import annotations

import numpy as np

POP_NAMES = ("L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I")


def population_stats(steps, ids, pop_offsets, t_start_step, t_end_step, dt_ms=0.1,
                     bin_ms=2.0, corr_neurons=200, corr_seed=12345):
    """Statistics of the raster (steps, ids) over [t_start_step, t_end_step).

    Returns {pop: {"rate_hz", "cv_isi", "corr", "n_cv"}} with
      rate_hz  mean over the population's neurons of spikes / duration,
      cv_isi   mean over neurons with >= 3 spikes of std(ISI) / mean(ISI),
      corr     mean Pearson correlation over pairs of `corr_neurons` neurons
               (drawn with a fixed seed) of their spike counts in `bin_ms` bins,
               over pairs whose counts vary.
    """
    steps = np.asarray(steps, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    keep = (steps >= t_start_step) & (steps < t_end_step)
    steps, ids = steps[keep], ids[keep]
    dur_s = (t_end_step - t_start_step) * dt_ms * 1e-3
    out = {}
    rng = np.random.Generator(np.random.Philox(corr_seed))
    order = np.lexsort((steps, ids))
    steps_o, ids_o = steps[order], ids[order]
    bounds = np.searchsorted(ids_o, np.arange(pop_offsets[-1] + 1))
    bin_steps = int(round(bin_ms / dt_ms))
    nbins = (t_end_step - t_start_step) // bin_steps
    for a, name in enumerate(POP_NAMES):
        lo, hi = int(pop_offsets[a]), int(pop_offsets[a + 1])
        n = hi - lo
        counts = bounds[lo + 1:hi + 1] - bounds[lo:hi]
        rate = counts.sum() / (n * dur_s)
        cvs = []
        for i in range(lo, hi):
            s = steps_o[bounds[i]:bounds[i + 1]]
            if len(s) >= 3:
                isi = np.diff(s).astype(np.float64)
                cvs.append(isi.std() / isi.mean())
        pick = np.sort(rng.choice(np.arange(lo, hi), size=min(corr_neurons, n), replace=False))
        mat = np.zeros((len(pick), nbins))
        for r, i in enumerate(pick):
            s = steps_o[bounds[i]:bounds[i + 1]]
            b = (s - t_start_step) // bin_steps
            b = b[b < nbins]
            np.add.at(mat[r], b, 1.0)
        var = mat.std(axis=1) > 0
        m = mat[var]
        corr = np.nan
        if len(m) >= 2:
            c = np.corrcoef(m)
            iu = np.triu_indices(len(m), 1)
            corr = float(c[iu].mean())
        out[name] = {"rate_hz": float(rate), "cv_isi": float(np.mean(cvs)) if cvs else float("nan"),
                     "corr": corr, "n_cv": len(cvs)}
    return out
