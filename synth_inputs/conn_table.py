"""Seeded stand-in for the microcircuit's 8x8 connection-probability table.

The published table of the layered microcircuit model is not part of this
repository; the simulator takes the table as a required input.  This stand-in
is synthetic and named as such.  Its recipe aims at the workload *shape* the
paper reports for the full model: 77,169 neurons, about 3e8 synapses (Sec. 2a)
and an inhibition-dominated, low-rate asynchronous state with tens of spikes
per 0.1 ms step (Sec. 2c).

Recipe (seeded by ``seed`` through numpy's Philox generator):
  * every post population b receives the same mean recurrent in-degree
    K_in = total_synapses / 77,169;
  * a fraction rho_b/(1+rho_b) of it comes from the four inhibitory
    populations, 1/(1+rho_b) from the four excitatory ones; rho_b rises
    linearly with the population's background in-degree K_ext from rho_lo (at
    the smallest K_ext) to rho_hi (at the largest), so that populations with
    stronger Poisson drive receive proportionally more inhibition (with the -4
    inhibitory weight factor, inhibition dominates everywhere);
  * within each class the in-degree is split over source populations in
    proportion to N_a * U(0.5, 1.5);
  * p_ab = 1 - exp(-k_ab / N_a), so that the fixed-total-number rule
    K = log(1-p)/log(1-1/(N_a N_b)) gives k_ab * N_b synapses.
Entries are in [0, 0.4]; the full-scale total is ~3e8.
"""
from __future__ import annotations

import numpy as np

POP_NAMES = ("L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I")
FULL_SIZE = (20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948)
K_EXT = (1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100)
STANDIN_SEED = 20190918
_EXC = np.array([1, 0, 1, 0, 1, 0, 1, 0], dtype=bool)


RHO_DEFAULT = (0.4, 0.8)


def standin_conn_table(seed: int = STANDIN_SEED, rho=RHO_DEFAULT, total_synapses: float = 3.0e8):
    """Return a float64 array [8, 8]: entry [a, b] = pre population a -> post b."""
    rng = np.random.Generator(np.random.Philox(seed))
    n = np.asarray(FULL_SIZE, dtype=np.float64)
    k_in = total_synapses / n.sum()
    jitter = rng.uniform(0.5, 1.5, size=(8, 8))
    lo, hi = (rho, rho) if np.isscalar(rho) else rho
    kext = np.asarray(K_EXT, dtype=np.float64)
    rho_b = lo + (hi - lo) * (kext - kext.min()) / (kext.max() - kext.min())
    p = np.zeros((8, 8))
    for b in range(8):
        r = rho_b[b]
        for cls, share in ((_EXC, 1.0 / (1.0 + r)), (~_EXC, r / (1.0 + r))):
            wgt = n[cls] * jitter[cls, b]
            k_ab = k_in * share * wgt / wgt.sum()
            p[cls, b] = 1.0 - np.exp(-k_ab / n[cls])
    assert p.min() >= 0.0 and p.max() <= 0.4
    return p


def standin_description(seed: int = STANDIN_SEED, rho=RHO_DEFAULT):
    lo, hi = (rho, rho) if np.isscalar(rho) else rho
    return (f"synthetic stand-in connection table (seed {seed}, inhibitory/excitatory "
            f"in-degree ratio {lo}..{hi} rising with K_ext)")
