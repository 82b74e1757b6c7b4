"""Pins of oracle/stats.py (the spike-train statistics of Sec. 4b: population
firing rate, CV of the inter-spike interval, correlation of binned counts) on
hand-built rasters whose statistics are known in closed form.  The statistics
are computed the same way for the FP64 reference and for the GPU runs, so a
mistake in them would cancel in that comparison; these tests catch it here."""
import math

import numpy as np
import pytest

from oracle.stats import POP_NAMES, population_stats

DT_MS = 0.1


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def _raster(trains):
    """trains: {neuron id: list of steps} -> (steps, ids) sorted by (step, id)."""
    pairs = sorted((int(s), int(i)) for i, ss in trains.items() for s in ss)
    if not pairs:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    st, ids = zip(*pairs)
    return np.array(st, np.int64), np.array(ids, np.int64)


def test_regular_train_rate_and_zero_cv():
    # population 0: 4 neurons; neuron 0 fires every 50 steps (200 Hz at dt 0.1 ms),
    # the other three are silent.  Window [1000, 11000): exactly 200 spikes of neuron 0.
    sizes = [4, 1, 1, 1, 1, 1, 1, 1]
    st, ids = _raster({0: range(0, 12000, 50)})
    out = population_stats(st, ids, _offsets(sizes), 1000, 11000, dt_ms=DT_MS)
    dur_s = 10000 * DT_MS * 1e-3
    # silent neurons count in the denominator of the population rate
    assert out["L23E"]["rate_hz"] == pytest.approx(200 / (4 * dur_s), rel=1e-12)
    assert out["L23E"]["cv_isi"] == 0.0
    assert out["L23E"]["n_cv"] == 1                   # silent neurons have no CV
    assert out["L23I"]["rate_hz"] == 0.0 and out["L23I"]["n_cv"] == 0 and math.isnan(out["L23I"]["cv_isi"])


def test_window_edges_exact():
    # spikes exactly at the first step of the window are kept, at the end step dropped
    sizes = [1] * 8
    st, ids = _raster({0: [999, 1000, 1500, 1999, 2000]})
    out = population_stats(st, ids, _offsets(sizes), 1000, 2000, dt_ms=DT_MS)
    assert out["L23E"]["rate_hz"] == pytest.approx(3 / (1000 * DT_MS * 1e-3), rel=1e-12)
    assert out["L23E"]["n_cv"] == 1
    # ISIs 500, 499: population standard deviation (ddof 0) over the mean
    isi = np.array([500.0, 499.0])
    assert out["L23E"]["cv_isi"] == pytest.approx(0.5 / 499.5, rel=1e-12)
    assert out["L23E"]["cv_isi"] == pytest.approx(isi.std() / isi.mean(), rel=1e-12)


def test_cv_three_spike_closed_form():
    # ISIs 10 and 20 steps: mean 15, standard deviation 5 (ddof 0) -> CV 1/3;
    # ddof 1 would give sqrt(50)/15 = 0.471
    sizes = [1] * 8
    st, ids = _raster({2: [100, 110, 130]})           # neuron 2 is population L4E (index 2)
    out = population_stats(st, ids, _offsets(sizes), 0, 1000, dt_ms=DT_MS)
    assert out["L4E"]["cv_isi"] == pytest.approx(1.0 / 3.0, rel=1e-12)
    assert out["L4E"]["n_cv"] == 1
    # two spikes give one ISI only: no CV for that neuron
    st, ids = _raster({2: [100, 110]})
    out = population_stats(st, ids, _offsets(sizes), 0, 1000, dt_ms=DT_MS)
    assert out["L4E"]["n_cv"] == 0


def test_cv_mean_over_neurons():
    # population L23E of 3 neurons: CVs 0 (regular), 1/3 (10, 20) and silent -> mean 1/6
    sizes = [3, 1, 1, 1, 1, 1, 1, 1]
    st, ids = _raster({0: [0, 10, 20, 30], 1: [5, 15, 35]})
    out = population_stats(st, ids, _offsets(sizes), 0, 1000, dt_ms=DT_MS)
    assert out["L23E"]["cv_isi"] == pytest.approx(1.0 / 6.0, rel=1e-12)
    assert out["L23E"]["n_cv"] == 2


def test_poisson_train_cv_near_one():
    # Bernoulli spikes with probability q per step: geometric ISIs, CV sqrt(1 - q)
    rng = np.random.default_rng(11)
    q = 0.002
    steps = np.flatnonzero(rng.random(2_000_000) < q)
    sizes = [1] * 8
    st, ids = _raster({0: steps})
    out = population_stats(st, ids, _offsets(sizes), 0, 2_000_000, dt_ms=DT_MS)
    n = len(steps) - 1
    assert abs(out["L23E"]["cv_isi"] - math.sqrt(1 - q)) < 3 / math.sqrt(n)
    assert out["L23E"]["rate_hz"] == pytest.approx(len(steps) / 200.0, rel=1e-12)


def test_correlation_identical_and_opposite():
    # 2 ms bins = 20 steps from the window start.  Neurons 0 and 1 (population
    # L23E) fire identically -> correlation 1.  Neurons 2 and 3 (L23I) fire in
    # alternating bins -> counts (1, 0, 1, 0, ...) and (0, 1, 0, 1, ...): -1.
    sizes = [2, 2, 1, 1, 1, 1, 1, 1]
    t0, nb = 100, 50
    rng = np.random.default_rng(2)
    same = [t0 + 20 * b + int(rng.integers(0, 20)) for b in range(nb) if rng.random() < 0.5]
    even = [t0 + 20 * b + 3 for b in range(0, nb, 2)]
    odd = [t0 + 20 * b + 17 for b in range(1, nb, 2)]
    st, ids = _raster({0: same, 1: same, 2: even, 3: odd})
    out = population_stats(st, ids, _offsets(sizes), t0, t0 + 20 * nb, dt_ms=DT_MS, bin_ms=2.0)
    assert out["L23E"]["corr"] == pytest.approx(1.0, abs=1e-12)
    assert out["L23I"]["corr"] == pytest.approx(-1.0, abs=1e-12)


def test_correlation_bins_start_at_window():
    # A spike at window start + 19 falls in bin 0, at + 20 in bin 1: neurons with
    # spikes in the same bins correlate at 1 only if the bins begin at the window
    # start (a bin grid from step 0 would split them at t0 = 110).
    sizes = [2, 1, 1, 1, 1, 1, 1, 1]
    t0, nb = 110, 40
    a = [t0 + 20 * b for b in range(0, nb, 3)]
    b_ = [t0 + 20 * b + 19 for b in range(0, nb, 3)]
    st, ids = _raster({0: a, 1: b_})
    out = population_stats(st, ids, _offsets(sizes), t0, t0 + 20 * nb, dt_ms=DT_MS, bin_ms=2.0)
    assert out["L23E"]["corr"] == pytest.approx(1.0, abs=1e-12)


def test_correlation_excludes_constant_rows_and_independent_near_zero():
    # population L23E: 60 neurons with independent Bernoulli bins, plus 20 silent;
    # silent rows have no variance and are excluded; the mean pairwise correlation
    # of independent trains is 0 within its sampling error.
    sizes = [80, 1, 1, 1, 1, 1, 1, 1]
    rng = np.random.default_rng(5)
    nb = 4000
    trains = {i: [20 * b + 5 for b in range(nb) if rng.random() < 0.3] for i in range(60)}
    st, ids = _raster(trains)
    out = population_stats(st, ids, _offsets(sizes), 0, 20 * nb, dt_ms=DT_MS, bin_ms=2.0, corr_neurons=80)
    # each pair's correlation has standard deviation ~1/sqrt(nb); uncentred
    # products would give ~0.3 instead
    assert abs(out["L23E"]["corr"]) < 3 / math.sqrt(nb)
    assert np.isfinite(out["L23E"]["corr"])


def test_population_names_and_order():
    assert POP_NAMES == ("L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I")
    sizes = [1, 2, 3, 4, 5, 6, 7, 8]
    off = _offsets(sizes)
    # one spike of the last neuron of each population
    st, ids = _raster({int(off[a + 1] - 1): [10 + a] for a in range(8)})
    out = population_stats(st, ids, off, 0, 10000, dt_ms=DT_MS)
    for a, p in enumerate(POP_NAMES):
        assert out[p]["rate_hz"] == pytest.approx(1 / (sizes[a] * 1.0), rel=1e-12)
