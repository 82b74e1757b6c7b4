"""Brute-force reference for tiny hand-made networks -- pure Python loops.

TEST INFRASTRUCTURE ONLY.  It pins the C oracle: on explicit networks of a few
neurons it recomputes everything the oracle does (Philox draws, Poisson
thresholds, weight quantisation, the exact-integration update, the delay
buffers) with Python integers, Python floats (IEEE double) and numpy float32
scalars (IEEE single, one rounding per operation, no fused multiply-add).

Model: Eq. 1 of Rhodes et al. (arXiv 1909.08665, Sec. 2a) integrated exactly
over a step; input buffers with one slot per future step, the current slot
consumed each step (Sec. 3a(ii)); Poisson background count times the background
weight added to the step's input (Sec. 3a(ii)).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

MASK64 = (1 << 64) - 1
KMAX = 24


def philox4x64_10(ctr, key):
    """Philox4x64-10 (Salmon et al., SC'11) on Python integers."""
    c = [int(x) & MASK64 for x in ctr]
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    for _ in range(10):
        prod_a = 0xD2E7470EE14C6C93 * c[0]
        prod_b = 0xCA5A826395121157 * c[2]
        c = [(prod_b >> 64) ^ c[1] ^ k0, prod_b & MASK64, (prod_a >> 64) ^ c[3] ^ k1, prod_a & MASK64]
        k0 = (k0 + 0x9E3779B97F4A7C15) & MASK64
        k1 = (k1 + 0xBB67AE8584CAA73B) & MASK64
    return c


def round_to_format_exact(x: float, frac_bits: int, emin: int) -> float:
    """Nearest value of a binary format (ties to even), by exact rational search."""
    if x == 0.0:
        return 0.0
    q = Fraction(x)
    a = abs(q)
    e = emin
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    quantum = Fraction(2) ** (e - frac_bits)
    m = a / quantum
    lo = math.floor(m)
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    r = float(lo * quantum)
    return -r if x < 0 else r


def poisson_thresholds(lam: float):
    out = []
    term = math.exp(-lam)
    cdf = term
    for k in range(KMAX):
        if k:
            term = (term * lam) / k
            cdf = cdf + term
        out.append(1 << 32 if cdf >= 1.0 else int(math.floor(math.ldexp(cdf, 32))))
    return out


class BruteNet:
    """Explicit network: pop_sizes[8], synapse lists (pre, post, w pA, d steps)."""

    def __init__(self, pop_sizes, pre, post, w, d, *, seed=1, fp64=False, wfmt=0, poisson_on=True,
                 init_zero=False, i_dc=None, k_ext=None, full_params=None, relaxed=None):
        p = dict(nu_bg=8.0, dt=0.1, tau_m=10.0, c_m=250.0, tau_s=0.5, t_ref=2.0, theta=15.0, w_ext=87.8)
        if full_params:
            p.update(full_params)
        self.p = p
        self.seed = int(seed)
        self.fp64 = fp64
        self.poisson_on = poisson_on
        self.pop_of = []
        for a, sz in enumerate(pop_sizes):
            self.pop_of += [a] * int(sz)
        self.N = len(self.pop_of)
        k_ext = k_ext if k_ext is not None else (1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100)
        i_dc = i_dc if i_dc is not None else [0.0] * 8

        def stored(wv):
            if wfmt == 1:
                return round_to_format_exact(wv, 10, -14)
            if wfmt == 2:
                return round_to_format_exact(wv, 7, -126)
            return wv

        self.syn = []      # (pre, post, wq, w64, d)
        for a_, b_, w_, d_ in zip(pre, post, w, d):
            self.syn.append((int(a_), int(b_), int(round(stored(float(w_)) * 256.0)), float(w_), int(d_)))
        self.wq_ext = int(round(stored(p["w_ext"]) * 256.0))   # round(): ties to even, as rint
        maxd = max([s[4] for s in self.syn], default=1)
        R = 2
        while R < maxd + 1:
            R *= 2
        self.R = R

        dt = p["dt"]
        self.P22 = math.exp(-dt / p["tau_m"])
        self.P11 = math.exp(-dt / p["tau_s"])
        self.P21 = ((p["tau_m"] * p["tau_s"]) / (p["c_m"] * (p["tau_m"] - p["tau_s"]))) * (self.P22 - self.P11)
        self.P20 = (p["tau_m"] / p["c_m"]) * (1.0 - self.P22)
        self.ref = int(round(p["t_ref"] / dt))
        self.cdc = [self.P20 * float(x) for x in i_dc]
        self.thr = [poisson_thresholds(((p["nu_bg"] * k_ext[a]) * dt) * 1e-3) for a in range(8)]

        f32 = np.float32
        self.u, self.I = [], []
        for i in range(self.N):
            i0 = 0.0
            if relaxed is not None:
                u0, i0 = self._relaxed(i, self.pop_of[i], relaxed)
            elif init_zero:
                u0 = 0.0
            else:
                u0 = p["theta"] * ((philox4x64_10((i, 0, 0, 3), (self.seed, 0))[0] >> 11) * 2.0 ** -53)
            self.u.append(u0 if fp64 else f32(u0))
            self.I.append(i0 if fp64 else f32(i0))
        self.refr = [0] * self.N
        self.ring = [[0.0 if fp64 else 0 for _ in range(self.N)] for _ in range(R)]
        self.step = 0
        self.spikes = []

    def _relaxed(self, i, a, r):
        """Relaxed start: I ~ N(i_mean, i_sd) from the first normal pair's second
        member; u ~ N(u_mean, u_sd) restricted to u < theta with acceptance
        1 - exp(-2 (theta - u)(theta - u_mean) / u_sd^2) (the normal density minus
        its image in the threshold), trying blocks (i, 1 + k, 0, 3) in turn."""
        mu, sd, th = r["u_mean"][a], r["u_sd"][a], self.p["theta"]
        two_pi = 6.283185307179586
        cur = 0.0
        for k in range(64):
            x = philox4x64_10((i, 1 + k, 0, 3), (self.seed, 0))
            rad = math.sqrt(-2.0 * math.log(((x[0] >> 11) + 1) * 2.0 ** -53))
            phi = two_pi * ((x[1] >> 11) * 2.0 ** -53)
            z1 = rad * math.cos(phi)
            if k == 0:
                cur = r["i_mean"][a] + r["i_sd"][a] * (rad * math.sin(phi))
            v = mu + sd * z1
            accept = 1.0 - math.exp(-2.0 * (th - v) * (th - mu) / (sd * sd))
            if v < th and (x[2] >> 11) * 2.0 ** -53 < accept:
                return v, cur
        return 0.0, cur

    def poisson(self, n, i):
        """Count for neuron i at step n: 32-bit half i mod 8 of the block
        (n, i // 8, 0, 2), halves taken high then low of each 64-bit word."""
        block = philox4x64_10((n, i // 8, 0, 2), (self.seed, 0))
        halves = [h for w in block for h in (w >> 32, w & 0xFFFFFFFF)]
        v = halves[i % 8]
        return sum(1 for t in self.thr[self.pop_of[i]] if v >= t)

    def run(self, steps):
        f32 = np.float32
        p = self.p
        for _ in range(steps):
            n = self.step
            slot = n % self.R
            fired = []
            for i in range(self.N):
                raw = self.ring[slot][i]
                self.ring[slot][i] = 0.0 if self.fp64 else 0
                k = self.poisson(n, i) if self.poisson_on else 0
                pop = self.pop_of[i]
                if self.fp64:
                    x = raw + k * p["w_ext"]
                    u, I = self.u[i], self.I[i]
                    if self.refr[i] > 0:
                        self.refr[i] -= 1
                    else:
                        u = self.P22 * u + self.P21 * I
                        if self.cdc[pop] != 0.0:
                            u = u + self.cdc[pop]
                    I = self.P11 * I + x
                    spk = u > p["theta"]
                    if spk:
                        u = 0.0
                else:
                    q = int(raw) + k * self.wq_ext
                    x = f32(q) * f32(0.00390625)
                    u, I = self.u[i], self.I[i]
                    if self.refr[i] > 0:
                        self.refr[i] -= 1
                    else:
                        u = f32(self.P22) * u + f32(self.P21) * I
                        c = f32(self.cdc[pop])
                        if c != f32(0.0):
                            u = u + c
                    I = f32(self.P11) * I + x
                    spk = u > f32(p["theta"])
                    if spk:
                        u = f32(0.0)
                if spk:
                    self.refr[i] = self.ref
                    fired.append(i)
                self.u[i], self.I[i] = u, I
            for i in fired:
                self.spikes.append((n, i))
                for (a_, b_, wq, w64, d_) in self.syn:
                    if a_ == i:
                        s = (n + d_) % self.R
                        self.ring[s][b_] += w64 if self.fp64 else wq
            self.step += 1

    def inject(self, ids):
        """Deliver the rows of the listed neurons as if they had spiked in the
        step before the current one: weight into slot (step - 1 + delay)."""
        n = self.step - 1
        for i in ids:
            i = int(i)
            if not 0 <= i < self.N:
                raise ValueError("neuron id out of range")
            for (a_, b_, wq, w64, d_) in self.syn:
                if a_ == i:
                    s = (n + d_) % self.R
                    self.ring[s][b_] += w64 if self.fp64 else wq
