"""Seeded stand-in for the microcircuit's 8x8 connection-probability table.

The published table of the layered microcircuit model is not part of this
repository; the simulator takes the table as a required input.  This stand-in
is synthetic and named as such.  Its recipe aims at the workload *shape* the
paper reports for the full model -- 77,169 neurons, about 3e8 synapses
(Sec. 2a), and an inhibition-dominated, low-rate asynchronous irregular state
with about 25 spikes per 0.1 ms step and peaks of tens (Sec. 2c) -- in which
per-population statistics are stable from run to run, so that a change of
arithmetic can be judged by them (Sec. 4b).

Recipe (the only random numbers come from numpy's Philox generator, `seed`):
  * every post population b receives the same mean recurrent in-degree
    K = total_synapses / 77,169;
  * its excitatory part K_E(b) is split over the four excitatory populations in
    proportion to N_a * U(1 - jitter, 1 + jitter), the inhibitory part K_I(b)
    likewise over the four inhibitory ones;
  * K_I(b) = K - K_E(b) is set so that, with every population firing at a
    common rate nu, the mean input current of b equals mu (pA), below the
    rheobase theta * C / tau_m = 375 pA, so that firing is driven by
    fluctuations:
        K_ext(b) nu_bg w tau_syn + nu tau_syn (K_E(b) wbar_E(b) - K_I(b) 4 w) = mu,
    with w = 87.8 pA, the inhibitory weight -4 w, and wbar_E(b) the mean
    excitatory weight onto b (the L4E -> L2/3E mean is doubled);
  * p_ab = 1 - exp(-k_ab / N_a), so that the fixed-total-number rule
    K = log(1-p)/log(1-1/(N_a N_b)) gives k_ab * N_b synapses.
The defaults (nu = 3 Hz, mu = 300 pA, jitter 0.2) were chosen among nu in
{2, 2.5, 3, 3.3, 5} Hz, mu in {150 .. 360} pA and jitter in {0, 0.1, 0.2, 0.5}
by full-scale runs: jitter 0.5 gives bursting or silent populations; the
others are asynchronous, and these defaults give 24 spikes per step, every
population between 2.3 and 4.5 Hz, and run-to-run spreads of population rates
and CV-ISI below 1 %.  Entries are in [0, 0.4]; the full-scale total is ~3e8.
"""
from __future__ import annotations

import numpy as np

POP_NAMES = ("L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I")
FULL_SIZE = (20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948)
K_EXT = (1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100)
STANDIN_SEED = 20190918
_EXC = np.array([1, 0, 1, 0, 1, 0, 1, 0], dtype=bool)

STANDIN_RATE_HZ = 3.0
STANDIN_MEAN_INPUT_PA = 300.0
STANDIN_JITTER = 0.2


def standin_conn_table(seed: int = STANDIN_SEED, rate_hz: float = STANDIN_RATE_HZ,
                       mean_input_pa: float = STANDIN_MEAN_INPUT_PA, jitter: float = STANDIN_JITTER,
                       total_synapses: float = 3.0e8):
    """Return a float64 array [8, 8]: entry [a, b] = pre population a -> post b."""
    rng = np.random.Generator(np.random.Philox(seed))
    shares = rng.uniform(1.0 - jitter, 1.0 + jitter, size=(8, 8))
    n = np.asarray(FULL_SIZE, dtype=np.float64)
    k_in = total_synapses / n.sum()
    w, tau_syn_s, nu_bg = 87.8, 0.5e-3, 8.0
    mu_ext = np.asarray(K_EXT, dtype=np.float64) * nu_bg * w * tau_syn_s
    p = np.zeros((8, 8))
    for b in range(8):
        we = n[_EXC] * shares[_EXC, b]
        frac_e = we / we.sum()
        wbar_e = w * (1.0 + (frac_e[1] if b == 0 else 0.0))      # L4E (2nd excitatory) -> L2/3E doubled
        k_i = (mu_ext[b] + tau_syn_s * rate_hz * k_in * wbar_e - mean_input_pa) / (tau_syn_s * rate_hz * (wbar_e + 4 * w))
        k_i = min(max(k_i, 0.05 * k_in), 0.95 * k_in)
        k_e = k_in - k_i
        wi = n[~_EXC] * shares[~_EXC, b]
        p[_EXC, b] = 1.0 - np.exp(-(k_e * frac_e) / n[_EXC])
        p[~_EXC, b] = 1.0 - np.exp(-(k_i * wi / wi.sum()) / n[~_EXC])
    assert p.min() >= 0.0 and p.max() <= 0.4
    return p


def standin_description(seed: int = STANDIN_SEED):
    return (f"synthetic stand-in connection table (seed {seed}; every population's mean input "
            f"{STANDIN_MEAN_INPUT_PA:g} pA at a common {STANDIN_RATE_HZ:g} Hz, shares jittered "
            f"+-{STANDIN_JITTER:g})")
