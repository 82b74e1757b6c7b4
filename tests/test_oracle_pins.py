"""Pins of the CPU oracle against facts fixed outside it: numpy's Philox, scipy's
Poisson CDF, exact decimal arithmetic, closed-form solutions of Eq. 1
(Rhodes et al., arXiv 1909.08665, Sec. 2a), the defining property of the
fixed-total-number connection rule, distribution moments and invariants."""
import math
from decimal import ROUND_FLOOR, Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

from oracle import brute
from oracle import oracle as O

M64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------
def _numpy_block(ctr, key):
    """Philox4x64-10 block for `ctr` via numpy (numpy increments before use)."""
    c = sum(int(x) << (64 * k) for k, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * k)) & M64 for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 2, 3, 4), (5, 0)),
    ((123456789, 77168, 0, 2), (20190918, 0)),
    ((M64, M64, 0, 1), (M64, 0)),
    ((0, 63, 0, 1), (1, 0)),
    ((99999, 5, 0, 3), (2**63 + 7, 0)),
])
def test_philox_matches_numpy(ctr, key):
    expect = _numpy_block(ctr, key)
    assert [int(x) for x in O.philox(ctr, key)] == expect
    assert brute.philox4x64_10(ctr, key) == expect


# ---------------------------------------------------------------------------
# Reduced-precision rounding
# ---------------------------------------------------------------------------
def test_fp16_rounding_matches_numpy():
    rng = np.random.default_rng(3)
    xs = list(rng.normal(0, 200, 20000)) + list(rng.uniform(-1000, 1000, 20000))
    xs += [87.8, -351.2, 175.6, 65504.0, 2.0**-24, 3 * 2.0**-25, 1.0 + 2.0**-11, 1.0 + 3 * 2.0**-11]
    for x in xs:
        assert O.round_fp16(x) == float(np.float16(x)), x


def test_bf16_rounding_matches_exact_rational():
    rng = np.random.default_rng(4)
    xs = list(rng.normal(0, 200, 3000)) + [87.8, -351.2, 175.6, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -(1.0 + 2.0**-8)]
    for x in xs:
        assert O.round_bf16(x) == brute.round_to_format_exact(float(x), 7, -126), x


def test_background_weight_quantisation():
    # 87.8 pA in units of 1/256 pA: FP32 store rint(87.8*256); FP16 87.8125; BF16 88.0
    for wfmt, expect in ((O.W_FP32, 22477), (O.W_FP16, 22480), (O.W_BF16, 22528)):
        net = O.OracleNet.build_explicit([1, 0, 0, 0, 0, 0, 0, 0], [], [], [], [],
                                         params=O.default_params(wfmt=wfmt))
        assert net.wq_ext() == expect


# ---------------------------------------------------------------------------
# Step constants (exact integration of Eq. 1)
# ---------------------------------------------------------------------------
def test_propagator_constants_exact():
    getcontext().prec = 60
    dt, tm, ts, cm = Decimal("0.1"), Decimal(10), Decimal("0.5"), Decimal(250)
    p22 = (-dt / tm).exp()
    p11 = (-dt / ts).exp()
    p21 = tm * ts / (cm * (tm - ts)) * (p22 - p11)
    p20 = tm / cm * (1 - p22)
    net = O.OracleNet.build_explicit([1, 0, 0, 0, 0, 0, 0, 0], [], [], [], [])
    c = net.constants()
    for name, exact in (("P22", p22), ("P11", p11), ("P21", p21), ("P20", p20)):
        assert abs(c[name] - float(exact)) <= 1e-13 * float(exact), name  # 1 - P22 cancels ~2 digits
        assert c[name + "f"] == np.float32(float(exact)), name
    bits = {k: int(np.float32(c[k]).view(np.uint32)) for k in ("P22f", "P11f", "P21f", "P20f")}
    assert bits == {"P22f": 0x3F7D73E8, "P11f": 0x3F519857, "P21f": 0x39BD188B, "P20f": 0x39D0AB8C}


# ---------------------------------------------------------------------------
# Poisson background
# ---------------------------------------------------------------------------
def test_poisson_thresholds_vs_scipy():
    net = O.OracleNet.build_explicit([1] * 8, [], [], [], [])
    for a, kext in enumerate(O.K_EXT):
        lam = 8.0 * kext * 1e-4
        T = net.poisson_table(a).astype(np.float64)
        ref = np.floor(stats.poisson.cdf(np.arange(O.KMAX), lam) * 2.0**32)
        assert np.all(np.abs(T - ref) <= 2), a
        assert np.all(np.diff(T) >= 0)
        assert T[-1] >= 2.0**32 - 2


def test_poisson_counts_distribution():
    net = O.OracleNet.build_explicit([1] * 8, [], [], [], [])
    for a in (0, 6):                      # lambda = 1.28 and 2.32
        lam = 8.0 * O.K_EXT[a] * 1e-4
        ks = np.array([net.poisson_count(n, a) for n in range(60000)])
        assert abs(ks.mean() - lam) < 5 * math.sqrt(lam / len(ks))
        kmax = 8
        obs = np.bincount(np.minimum(ks, kmax), minlength=kmax + 1)
        pmf = stats.poisson.pmf(np.arange(kmax), lam)
        exp = np.append(pmf, 1 - pmf.sum()) * len(ks)
        chi2 = ((obs - exp) ** 2 / exp).sum()
        assert stats.chi2.sf(chi2, kmax) > 1e-4


def test_poisson_counts_independent_within_a_block():
    """Eight neurons share one Philox block per step (one 32-bit half each):
    their counts must be uncorrelated and individually Poisson."""
    net = O.OracleNet.build_explicit([16, 0, 0, 0, 0, 0, 0, 0], [], [], [], [])
    lam = 8.0 * O.K_EXT[0] * 1e-4
    steps = 20000
    k = np.array([[net.poisson_count(n, i) for i in range(16)] for n in range(steps)], dtype=np.float64)
    assert np.all(np.abs(k.mean(axis=0) - lam) < 5 * math.sqrt(lam / steps))
    c = np.corrcoef(k.T)
    off = c[~np.eye(16, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / math.sqrt(steps)


# ---------------------------------------------------------------------------
# Single-neuron closed forms
# ---------------------------------------------------------------------------
def _psp_net(mode, w=87.8, d=1):
    p = O.default_params(mode=mode, poisson_on=False, init_mode=1)
    net = O.OracleNet.build_explicit([2, 0, 0, 0, 0, 0, 0, 0], [0], [1], [w], [d], params=p)
    net.set_state(u=np.array([16.0, 0.0]))        # neuron 0 crosses threshold at step 0
    return net


@pytest.mark.parametrize("mode,tol", [(O.FP64, 1e-12), (O.MIRROR, 3e-6)])
def test_psp_shape_closed_form(mode, tol):
    """PSP of Eq. 1 for one input w at t=0: (w/C) tm ts/(tm-ts) (e^-t/tm - e^-t/ts)."""
    w, d = 87.8, 3
    net = _psp_net(mode, w, d)
    net.run(d + 1)                                 # the input enters I at step d
    us = []
    for _ in range(120):
        net.run(1)
        us.append(net.state()[0][1])
    wv = w if mode == O.FP64 else round(w * 256) / 256
    t = np.arange(1, 121) * 0.1
    closed = wv / 250.0 * (10 * 0.5 / 9.5) * (np.exp(-t / 10) - np.exp(-t / 0.5))
    peak = closed.max()
    assert np.max(np.abs(np.array(us) - closed)) <= tol * peak
    j = int(np.argmax(us))
    assert j + 1 == 16                              # discrete peak at 1.6 ms after arrival
    assert abs(peak - 0.1499775) < 1e-6 * (1 if mode == O.FP64 else 10)


def _fi_isi_closed(i_pa):
    """Steps between spikes under constant current: REF + first k with
    R I (1 - e^{-k dt/tau_m}) > theta."""
    rI = 0.04 * i_pa
    if rI <= 15.0:
        return None
    k = math.floor(math.log((rI - 15.0) / rI) / math.log(math.exp(-0.01))) + 1
    return 20 + k


@pytest.mark.parametrize("mode", [O.FP64, O.MIRROR])
def test_fi_curve_closed_form(mode):
    # exactly at rheobase (R I = theta) float rounding of the fixed point decides,
    # so the mirror is checked just below it
    silent = 375 if mode == O.FP64 else 370
    for i_pa, printed in ((400, 298), (500, 159), (600, 119), (800, 84), (1000, 68), (silent, None), (300, None)):
        expect = _fi_isi_closed(i_pa)
        assert expect == printed
        p = O.default_params(mode=mode, poisson_on=False, init_mode=1, i_dc=[i_pa] + [0] * 7)
        net = O.OracleNet.build_explicit([1, 0, 0, 0, 0, 0, 0, 0], [], [], [], [], params=p)
        net.run(3000)
        st, _ = net.spikes()
        if expect is None:
            assert len(st) == 0
            continue
        isi = np.diff(st)
        first = st[0] + 1
        if mode == O.FP64:
            assert first == expect - 20 and np.all(isi == expect), (i_pa, st[:4])
        else:
            assert abs(first - (expect - 20)) <= 1 and np.all(np.abs(isi - expect) <= 1)


# ---------------------------------------------------------------------------
# Connectivity
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def net2(conn_table):
    return O.OracleNet.build(11, 0.02, conn_table.reshape(64))


def _pairs(net):
    c = net.csr()
    pre = np.repeat(np.arange(net.N), np.diff(c["row_ptr"]))
    return c, pre, c["post"]


def test_population_sizes_2pct(net2):
    sizes = np.diff(net2.pop_offsets)
    assert sizes.tolist() == [414, 117, 438, 110, 97, 21, 288, 59]
    assert net2.N == 1544


def test_population_sizes_10pct(conn_table):
    """floor(N * 0.1 + 0.5): the ties 2191.5, 106.5 and 1439.5 round up."""
    net = O.OracleNet.build(3, 0.1, conn_table.reshape(64))
    assert np.diff(net.pop_offsets).tolist() == [2068, 583, 2192, 548, 485, 107, 1440, 295]
    assert net.N == 7718


def _k_exact(p, na, nb):
    """K = ln(1-p) / ln(1 - 1/(Na Nb)) in 60-digit decimal arithmetic, rounded to
    the nearest integer (halves up): independent of the oracle's double log1p."""
    if p == 0.0:
        return 0
    getcontext().prec = 60
    num = (Decimal(1) - Decimal(float(p))).ln()
    den = (Decimal(1) - Decimal(1) / (Decimal(int(na)) * Decimal(int(nb)))).ln()
    return int((num / den + Decimal("0.5")).to_integral_value(rounding=ROUND_FLOOR))


def _pair_counts(net):
    """Synapses per ordered population pair (pre a, post b), from the CSR."""
    import ctypes as C
    rp = np.zeros(net.N + 1, dtype=np.int64)
    post = np.zeros(net.M, dtype=np.int32)
    O.lib().or_get_csr(net._h, rp.ctypes.data_as(C.c_void_p), post.ctypes.data_as(C.c_void_p), None, None, None)
    off = net.pop_offsets
    pop_of = np.repeat(np.arange(8), np.diff(off))
    k = np.zeros((8, 8), dtype=np.int64)
    for a in range(8):
        seg = post[rp[off[a]]:rp[off[a + 1]]]
        k[a] = np.bincount(pop_of[seg], minlength=8)
    return k


@pytest.mark.parametrize("scale", [0.02, 0.1, 1.0])
def test_synapse_count_per_pair_exact(conn_table, scale):
    """Each ordered pair (a, b) holds exactly K_ab = round(ln(1-p)/ln(1-1/(N_a N_b)))
    synapses (Sec. 2a: connections by probability; the fixed-total-number reading)."""
    net = O.OracleNet.build(1, scale, conn_table.reshape(64))
    sizes = np.diff(net.pop_offsets)
    got = _pair_counts(net)
    for a in range(8):
        for b in range(8):
            assert got[a, b] == _k_exact(conn_table[a, b], sizes[a], sizes[b]), (scale, a, b)
    assert net.M == got.sum()


def test_synapse_count_log1p_not_log():
    """N_a = N_b = 20683, p = 0.1: K = 45,071,805.02 -> 45,071,805 (a naive log of
    1 - 1/N^2 in double gives 45,071,804.37 -> 45,071,804)."""
    assert _k_exact(0.1, 20683, 20683) == 45071805
    conn = np.zeros(64)
    conn[0] = 0.1
    net = O.OracleNet.build(1, 1.0, conn)
    assert net.M == 45071805
    naive = math.log(1 - 0.1) / math.log(1 - 1 / (20683.0 * 20683.0))
    assert math.floor(naive + 0.5) == 45071804


def test_connection_rule_defining_property(net2, conn_table):
    """K uniform draws with replacement leave a fraction p of distinct pairs connected."""
    _, pre, post = _pairs(net2)
    off = net2.pop_offsets
    pa = np.searchsorted(off, pre, side="right") - 1
    pb = np.searchsorted(off, post, side="right") - 1
    sizes = np.diff(off)
    zs = []
    for a in range(8):
        for b in range(8):
            p = conn_table[a, b]
            sel = (pa == a) & (pb == b)
            pairs = int(sizes[a]) * int(sizes[b])
            distinct = len(np.unique(pre[sel].astype(np.int64) * net2.N + post[sel]))
            sd = math.sqrt(pairs * p * (1 - p))
            zs.append((distinct - p * pairs) / max(sd, 1e-9))
    zs = np.array(zs)
    assert np.all(np.abs(zs) < 5)
    assert abs(zs.mean()) < 0.6


def test_total_synapses_near_scale_squared(conn_table):
    net = O.OracleNet.build(3, 0.1, conn_table.reshape(64))
    assert abs(net.M / 3.0e6 - 1) < 0.02


def test_pre_post_marginals_uniform(net2):
    _, pre, post = _pairs(net2)
    off = net2.pop_offsets
    for a in range(8):
        lo, hi = off[a], off[a + 1]
        for ids in (pre, post):
            sel = ids[(ids >= lo) & (ids < hi)]
            obs = np.bincount(sel - lo, minlength=hi - lo)
            chi2 = ((obs - obs.mean()) ** 2 / obs.mean()).sum()
            assert stats.chi2.sf(chi2, hi - lo - 1) > 1e-5


def test_weight_and_delay_distributions(conn_table):
    net = O.OracleNet.build(5, 0.05, conn_table.reshape(64), O.default_params(mode=O.FP64))
    c, pre, post = _pairs(net)
    off = net.pop_offsets
    pa = np.searchsorted(off, pre, side="right") - 1
    pb = np.searchsorted(off, post, side="right") - 1
    w, d = c["w64"], c["d"].astype(int)
    exc = pa % 2 == 0
    l4_l23 = (pa == 2) & (pb == 0)
    for sel, mean, sd in ((exc & ~l4_l23, 87.8, 8.78), (l4_l23, 175.6, 8.78), (~exc, -351.2, 35.12)):
        x = w[sel]
        assert abs(x.mean() - mean) < 5 * sd / math.sqrt(len(x))
        assert abs(x.std() / sd - 1) < 5 / math.sqrt(2 * len(x))
    assert np.all(w[exc] >= 0) and np.all(w[~exc] <= 0)          # Dale's law
    for sel, mu, sg in ((exc, 1.5, 0.75), (~exc, 0.8, 0.4)):
        x = d[sel]
        # rint((mu + sg z)/dt) clipped to [1, 255]: exact pmf from the normal CDF
        ks = np.arange(1, 60)
        lo = np.where(ks == 1, -np.inf, (ks - 0.5) * 0.1)
        hi = (ks + 0.5) * 0.1
        pmf = stats.norm.cdf(hi, mu, sg) - stats.norm.cdf(lo, mu, sg)
        obs = np.bincount(x, minlength=60)[1:60]
        keep = pmf * len(x) > 20
        chi2 = ((obs[keep] - pmf[keep] * len(x)) ** 2 / (pmf[keep] * len(x))).sum()
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-5
        assert x.min() >= 1 and x.max() <= 255


def test_quantised_weights_match_formats(conn_table):
    ref = O.OracleNet.build(8, 0.02, conn_table.reshape(64), O.default_params(mode=O.FP64)).csr()
    for wfmt, rnd in ((O.W_FP32, lambda x: x), (O.W_FP16, lambda x: float(np.float16(x))),
                      (O.W_BF16, lambda x: brute.round_to_format_exact(x, 7, -126))):
        c = O.OracleNet.build(8, 0.02, conn_table.reshape(64), O.default_params(wfmt=wfmt)).csr()
        idx = np.random.default_rng(1).choice(len(c["wq"]), 500, replace=False)
        for j in idx:
            assert c["wq"][j] == round(rnd(ref["w64"][j]) * 256)
        if wfmt != O.W_FP32:                          # exact multiples of 1/256 pA
            vals = np.array([rnd(ref["w64"][j]) for j in idx])
            assert np.all(vals * 256 == np.round(vals * 256))


# ---------------------------------------------------------------------------
# Dynamics invariants
# ---------------------------------------------------------------------------
def test_split_run_identity(conn_table):
    a = O.OracleNet.build(21, 0.02, conn_table.reshape(64))
    b = O.OracleNet.build(21, 0.02, conn_table.reshape(64))
    a.run(300)
    b.run(100)
    b.run(37)
    b.run(163)
    sa, sb = a.spikes(), b.spikes()
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_refractory_and_event_accounting(conn_table):
    net = O.OracleNet.build(22, 0.02, conn_table.reshape(64))
    net.run(1500)
    st, ids = net.spikes()
    c = net.csr()
    outdeg = np.diff(c["row_ptr"])
    cnt = net.counters()
    assert cnt["spikes"] == len(st)
    assert cnt["events"] == int(outdeg[ids].sum())
    order = np.lexsort((st, ids))
    same = np.diff(ids[order]) == 0
    assert np.all(np.diff(st[order])[same] >= 21)     # 20 refractory steps + one update


def test_ring_holds_exactly_the_pending_deliveries(conn_table):
    net = O.OracleNet.build(23, 0.02, conn_table.reshape(64))
    T = 777
    net.run(T)
    st, ids = net.spikes()
    c = net.csr()
    pending = 0
    for s, i in zip(st, ids):
        r0, r1 = c["row_ptr"][i], c["row_ptr"][i + 1]
        dd = c["d"][r0:r1].astype(np.int64)
        pending += int(c["wq"][r0:r1][s + dd >= T].sum())
    assert net.ring_sum() == pending


# ---------------------------------------------------------------------------
# Brute force on tiny explicit networks
# ---------------------------------------------------------------------------
def _tiny_net(seed, n_per_pop=(3, 2, 3, 1, 2, 1, 2, 1), m=60):
    rng = np.random.default_rng(seed)
    N = sum(n_per_pop)
    off = np.concatenate([[0], np.cumsum(n_per_pop)])
    pre = rng.integers(0, N, m)
    post = rng.integers(0, N, m)
    pop = np.searchsorted(off, pre, side="right") - 1
    w = np.where(pop % 2 == 0, rng.normal(87.8, 8.78, m), rng.normal(-351.2, 35.12, m)) * 3
    d = rng.integers(1, 40, m)
    return list(n_per_pop), pre, post, w, d


@pytest.mark.parametrize("mode,wfmt", [(O.MIRROR, O.W_FP32), (O.MIRROR, O.W_FP16), (O.MIRROR, O.W_BF16),
                                       (O.FP64, O.W_FP32)])
def test_brute_force_equals_oracle(mode, wfmt):
    sizes, pre, post, w, d = _tiny_net(7 + wfmt + 3 * mode)
    p = O.default_params(mode=mode, wfmt=wfmt)
    orc = O.OracleNet.build_explicit(sizes, pre, post, w, d, params=p, seed=99)
    bf = brute.BruteNet(sizes, pre, post, w, d, seed=99, fp64=(mode == O.FP64), wfmt=wfmt)
    for chunk in (60, 90, 150):
        orc.run(chunk)
        bf.run(chunk)
    st, ids = orc.spikes()
    assert list(zip(st.tolist(), ids.tolist())) == bf.spikes
    assert len(bf.spikes) > 20
    u, I, r = orc.state()
    assert np.array_equal(u, np.array(bf.u, dtype=np.float64))
    assert np.array_equal(I, np.array(bf.I, dtype=np.float64))
    assert r.tolist() == bf.refr


def test_brute_force_dc_input_equals_oracle():
    sizes, pre, post, w, d = _tiny_net(31)
    i_dc = [420.0, 380.0, 500.0, 0.0, 650.0, 390.0, 0.0, 800.0]
    p = O.default_params(poisson_on=False, i_dc=i_dc)
    orc = O.OracleNet.build_explicit(sizes, pre, post, w, d, params=p, seed=5)
    bf = brute.BruteNet(sizes, pre, post, w, d, seed=5, poisson_on=False, i_dc=i_dc)
    orc.run(400)
    bf.run(400)
    st, ids = orc.spikes()
    assert list(zip(st.tolist(), ids.tolist())) == bf.spikes and len(bf.spikes) > 10


def test_brute_force_injection_equals_oracle():
    """External stimulation: the rows of listed neurons land in the slots of
    step (n - 1) + delay, as if they had spiked in the last step (Sec. 3a(ii))."""
    sizes, pre, post, w, d = _tiny_net(41)
    for mode in (O.MIRROR, O.FP64):
        p = O.default_params(mode=mode)
        orc = O.OracleNet.build_explicit(sizes, pre, post, w, d, params=p, seed=3)
        bf = brute.BruteNet(sizes, pre, post, w, d, seed=3, fp64=(mode == O.FP64))
        for k, ids in enumerate(([0, 3, 3, 7], [1, 2, 4, 5, 6, 14], [9])):
            orc.inject(ids)
            bf.inject(ids)
            orc.run(40 + 13 * k)
            bf.run(40 + 13 * k)
        st, ids_ = orc.spikes()
        assert list(zip(st.tolist(), ids_.tolist())) == bf.spikes and len(bf.spikes) > 5
        u, I, r = orc.state()
        assert np.array_equal(u, np.array(bf.u, dtype=np.float64))
        assert np.array_equal(I, np.array(bf.I, dtype=np.float64))
    with pytest.raises(RuntimeError):
        orc.inject([sum(sizes)])


def test_overflow_bound_exact_edge():
    """int32 input buffers: the build is refused when some neuron's incoming
    sum of |weight| (1/256 pA) plus the largest background contribution
    (24 x 22477) reaches 2^31, and accepted one unit below."""
    pk = 24 * 22477
    total = 2 ** 31 - pk                              # 2146944200 = 100 * 21469442
    assert total == 100 * 21469442
    sizes = [1, 0, 0, 0, 0, 0, 0, 0]
    pre = post = [0] * 100
    d = [1] * 100
    w_at = [21469442 / 256.0] * 100                   # exact in double
    with pytest.raises(RuntimeError, match="overflow bound"):
        O.OracleNet.build_explicit(sizes, pre, post, w_at, d)
    w_below = [21469442 / 256.0] * 99 + [21469441 / 256.0]
    net = O.OracleNet.build_explicit(sizes, pre, post, w_below, d)
    assert net.M == 100
    # the background term counts: without it the first network would fit
    p = O.default_params(w_ext_pa=0.0)
    assert O.OracleNet.build_explicit(sizes, pre, post, w_at, d, params=p).M == 100


def test_overflow_bound_microcircuit(conn_table):
    """Absurd weights in the microcircuit builder: refused by the oracle (and,
    in test_lib_host, by the library with MC_ERR_OVERFLOW_BOUND)."""
    p = O.default_params(w_mean_pa=1.5e4, w_sd_pa=10.0)
    with pytest.raises(RuntimeError, match="overflow bound"):
        O.OracleNet.build(1, 0.1, conn_table.reshape(64), p)
    # a tenth of that weight fits
    assert O.OracleNet.build(1, 0.1, conn_table.reshape(64), O.default_params(w_mean_pa=1.5e3)).M > 0


RELAXED = dict(u_mean=[5.0, 5.7, 5.1, 5.9, 5.5, 6.1, 3.4, 5.0], u_sd=[3.9, 3.8, 3.9, 3.7, 3.8, 3.6, 4.4, 3.9],
               i_mean=[355.0, 368.0, 354.0, 371.0, 367.0, 371.0, 344.0, 364.0],
               i_sd=[455.0, 450.0, 457.0, 446.0, 449.0, 457.0, 511.0, 451.0])


def _relaxed_params(mode=O.MIRROR, r=RELAXED):
    return O.default_params(mode=mode, init_mode=2, init_u_mean_mv=r["u_mean"], init_u_sd_mv=r["u_sd"],
                            init_i_mean_pa=r["i_mean"], init_i_sd_pa=r["i_sd"])


@pytest.mark.parametrize("mode", [O.MIRROR, O.FP64])
def test_relaxed_start_brute_force_equals_oracle(mode):
    """The relaxed initial state (init_mode 2) drawn by the oracle equals the
    brute-force draw, and the run from it too."""
    sizes, pre, post, w, d = _tiny_net(51)
    orc = O.OracleNet.build_explicit(sizes, pre, post, w, d, params=_relaxed_params(mode), seed=77)
    bf = brute.BruteNet(sizes, pre, post, w, d, seed=77, fp64=(mode == O.FP64), relaxed=RELAXED)
    u, I, r = orc.state()
    assert np.array_equal(u, np.array(bf.u, dtype=np.float64))
    assert np.array_equal(I, np.array(bf.I, dtype=np.float64))
    orc.run(200)
    bf.run(200)
    st, ids = orc.spikes()
    assert list(zip(st.tolist(), ids.tolist())) == bf.spikes


def test_relaxed_start_distribution():
    """u follows the normal density minus its image in the threshold (zero at
    theta, below it everywhere), I the normal: checked on 200,000 draws against
    the closed-form density and moments."""
    r = dict(u_mean=[5.0] * 8, u_sd=[4.0] * 8, i_mean=[350.0] * 8, i_sd=[450.0] * 8)
    net = O.OracleNet.build_explicit([25000] * 8, [], [], [], [], params=_relaxed_params(O.FP64, r), seed=3)
    u, I, _ = net.state()
    th, mu, sd = 15.0, 5.0, 4.0
    assert u.max() < th
    # I: normal moments
    assert abs(I.mean() - 350.0) < 5 * 450 / math.sqrt(len(I))
    assert abs(I.std() / 450.0 - 1) < 5 / math.sqrt(2 * len(I))
    # u: histogram against the image density phi(u; mu) - phi(u; 2 th - mu), normalised below th
    edges = np.linspace(-15.0, 15.0, 31)
    cdf = lambda x: stats.norm.cdf(x, mu, sd) - stats.norm.cdf(x, 2 * th - mu, sd)
    mass = np.diff(cdf(edges))
    mass[0] += cdf(edges[0])                                  # everything below the first edge
    mass /= cdf(th)
    obs = np.histogram(np.clip(u, edges[0], edges[-1]), bins=edges)[0]
    exp = mass * len(u)
    keep = exp > 20
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    # near the threshold the density vanishes: the top 0.5 mV holds far fewer than a plain normal would
    assert (u > th - 0.5).mean() < 0.25 * (stats.norm.cdf(th, mu, sd) - stats.norm.cdf(th - 0.5, mu, sd))
