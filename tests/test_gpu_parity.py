"""GPU parity of libmc against the oracle's FP32 mirror: identical synapse
stores, spike rasters and final state, element by element, on the same seeded
inputs.  Every call goes through the C ABI."""
import numpy as np
import pytest

import paper_1909_08665_amd as mc
from oracle import oracle as O
from synth_inputs import standin_conn_table

pytestmark = pytest.mark.gpu

WF = {mc.W_FP32: O.W_FP32, mc.W_FP16: O.W_FP16, mc.W_BF16: O.W_BF16}


def _say(*a):
    print("[case]", *a, flush=True)


def _oracle(seed, scale, conn, wfmt=mc.W_FP32, **kw):
    p = O.default_params(wfmt=WF[wfmt], **kw)
    return O.OracleNet.build(seed, scale, np.asarray(conn).reshape(64), p)


def _canon(c, n):
    """Rows sorted by (post, delay, weight): a canonical form of a CSR store."""
    rp = c["row_ptr"]
    pre = np.repeat(np.arange(n), np.diff(rp))
    order = np.lexsort((c["wq"], c["d"], c["post"], pre))
    return rp, c["post"][order], c["d"][order], c["wq"][order]


def _same_run(lib_net, orc, inst=0):
    st, ids = lib_net.spikes(inst)
    rs, rids = orc.spikes(clear=True)
    assert len(st) == len(rs), (len(st), len(rs))
    assert np.array_equal(st, rs) and np.array_equal(ids, rids)
    u, I, r = lib_net.state(inst)
    ru, rI, rr = orc.state()
    assert np.array_equal(u.astype(np.float64), ru)
    assert np.array_equal(I.astype(np.float64), rI)
    assert np.array_equal(r, rr)
    return len(st)


@pytest.fixture(scope="module")
def conn():
    return standin_conn_table()


@pytest.mark.parametrize("scale", [0.02, 0.1])
@pytest.mark.parametrize("wfmt", [mc.W_FP32, mc.W_FP16, mc.W_BF16])
def test_synapse_store_equals_oracle(conn, scale, wfmt):
    _say("csr", scale, wfmt)
    net = mc.Network.build(3, scale, conn, wfmt=wfmt)
    orc = _oracle(3, scale, conn, wfmt)
    n, m = net.size()
    assert (n, m) == (orc.N, orc.M)
    a, b = _canon(net.csr(), n), _canon(orc.csr(), n)
    for x, y in zip(a, b):
        assert np.array_equal(x.astype(np.int64), y.astype(np.int64))
    assert net.info()["ring_depth"] == orc.R


def test_initial_state_equals_oracle(conn):
    _say("init state")
    net = mc.Network.build(17, 0.05, conn)
    orc = _oracle(17, 0.05, conn)
    u, I, r = net.state()
    ru, rI, rr = orc.state()
    assert np.array_equal(u.astype(np.float64), ru) and not I.any() and not r.any()


def test_poisson_and_lif_without_synapses(conn):
    """No recurrent synapses: isolates the Poisson draw and the LIF update."""
    _say("poisson only")
    z = np.zeros(64)
    net = mc.Network.build(5, 0.05, z)
    orc = _oracle(5, 0.05, z)
    for chunk in (1, 7, 300):
        net.run(chunk)
        orc.run(chunk)
        assert _same_run(net, orc) >= 0
    assert net.counters()["poisson_events"] == orc.counters()["poisson_events"]


@pytest.mark.parametrize("seed,engine", [(1, mc.ENGINE_TILED), (2, mc.ENGINE_TILED), (3, mc.ENGINE_TILED),
                                         (1, mc.ENGINE_GRAPH)])
def test_raster_parity_2pct_one_second(conn, seed, engine):
    """Microcircuit at 2 % (1544 neurons, ~1.2e5 synapses), 1 s = 10^4 steps."""
    _say("2pct 1s seed", seed, "engine", engine)
    net = mc.Network.build(seed, 0.02, conn, engine=engine)
    assert net.info()["engine"] == engine
    orc = _oracle(seed, 0.02, conn)
    net.run(10000)
    orc.run(10000)
    nspk = _same_run(net, orc)
    assert nspk > 1000
    c, rc = net.counters(), orc.counters()
    for k in ("steps", "spikes", "events", "poisson_events", "max_spikes_per_step"):
        assert c[k] == rc[k], k


@pytest.mark.parametrize("wfmt", [mc.W_FP16, mc.W_BF16])
def test_raster_parity_reduced_precision(conn, wfmt):
    _say("2pct reduced precision", wfmt)
    net = mc.Network.build(4, 0.02, conn, wfmt=wfmt)
    orc = _oracle(4, 0.02, conn, wfmt)
    net.run(3000)
    orc.run(3000)
    assert _same_run(net, orc) > 100


def test_split_runs_identical(conn):
    _say("split runs")
    a = mc.Network.build(9, 0.02, conn)
    b = mc.Network.build(9, 0.02, conn)
    a.run(1234)
    for k in (1, 49, 50, 51, 333, 750):
        b.run(k)
    sa, sb = a.spikes(), b.spikes()
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("knobs", [dict(engine=mc.ENGINE_GRAPH, block=64, seg=64, deliver_grid=7, graph_chunk=1),
                                   dict(engine=mc.ENGINE_GRAPH, block=512, seg=512, deliver_grid=4096, graph_chunk=200),
                                   dict(engine=mc.ENGINE_GRAPH, block=128, seg=128, deliver_grid=300, graph_chunk=13),
                                   dict(engine=mc.ENGINE_TILED, tile=64),
                                   dict(engine=mc.ENGINE_TILED, tile=333),
                                   dict(engine=mc.ENGINE_TILED, tile=512),
                                   dict(engine=mc.ENGINE_TILED, tile=333, ring=2),
                                   dict(engine=mc.ENGINE_TILED, tile=2000, ring=2),
                                   dict(engine=mc.ENGINE_TILED, tile=4000, ring=2)])
def test_launch_configuration_invariance(conn, knobs):
    _say("launch knobs", knobs)
    net = mc.Network.build(12, 0.05, conn)
    net.set_launch(**knobs)
    orc = _oracle(12, 0.05, conn)
    net.run(1500)
    orc.run(1500)
    assert _same_run(net, orc) > 100


def test_recorder_larger_than_first_copy(conn):
    """Every neuron of a 10 % network starts above threshold: the first step
    records all 7,718 spikes, more than the entries the step kernel's launch
    has copied to the host with its head (sized from the spike rate so far,
    4,160 here), so the host copies the rest; the raster is still the
    oracle's, bit for bit."""
    _say("recorder larger than the first copy")
    net = mc.Network.build(17, 0.1, conn)
    orc = _oracle(17, 0.1, conn)
    u, _, _ = orc.state()
    u[:] = 16.0
    orc.set_state(u=u)
    net.set_state(u=u.astype(np.float32))
    net.run(1)
    orc.run(1)
    assert _same_run(net, orc) == len(u)
    net.run(300)
    orc.run(300)
    assert _same_run(net, orc) > 0


def test_more_tiles_than_compute_units(conn):
    """Tiles of 16 neurons at 10 % scale: 483 workgroups, two or more per
    compute unit, which the library then launches cooperatively so that all of
    them are resident at once; bit-exact against the oracle."""
    _say("more tiles than compute units")
    net = mc.Network.build(16, 0.1, conn)
    net.set_launch(engine=mc.ENGINE_TILED, tile=16)
    info = net.info()
    assert info["n_tiles"] > 256, info
    orc = _oracle(16, 0.1, conn)
    for chunk in (7, 993):
        net.run(chunk)
        orc.run(chunk)
    assert _same_run(net, orc) > 100


def test_tiling_beyond_lds_residency_is_refused(conn):
    """Full scale in tiles of 101 neurons: 765 workgroups of about 54 KB of LDS
    each, of which only two fit in a compute unit's 160 KB, so they cannot all
    be resident at once.  The tiling is refused at set-up (the occupancy
    query alone would have let it through, and the launch would then wait for
    workgroups that are never placed); 151-neuron tiles, two per CU, run."""
    _say("tiling beyond LDS residency")
    net = mc.Network.build(1, 1.0, conn)
    with pytest.raises(mc.MCError) as e:
        net.set_launch(engine=mc.ENGINE_TILED, tile=101, ring=1)
    assert e.value.code == -9 and "resident" in str(e.value)
    net.set_launch(engine=mc.ENGINE_TILED, tile=151, ring=1)
    assert net.info()["n_tiles"] == 512
    net.run(50)
    assert len(net.spikes()[0]) > 0


def test_tile_too_large_for_lds_is_refused(conn):
    _say("tile refusal")
    net = mc.Network.build(12, 0.05, conn)
    with pytest.raises(mc.MCError) as e:
        net.set_launch(engine=mc.ENGINE_TILED, tile=1024, ring=1)     # [64][1024] int32 ring > 160 KB
    assert e.value.code == -9
    net.set_launch(engine=mc.ENGINE_TILED, tile=1024)             # auto: ring moves to global memory
    assert net.info()["lds_ring"] == 0
    net.run(10)                                             # the previous engine still runs


def test_engine_switching_mid_run(conn):
    """Alternate engines and tile sizes between runs of one network."""
    _say("engine switching")
    net = mc.Network.build(31, 0.05, conn)
    orc = _oracle(31, 0.05, conn)
    for k, knobs in enumerate([dict(engine=mc.ENGINE_TILED, tile=128), dict(engine=mc.ENGINE_GRAPH),
                               dict(engine=mc.ENGINE_TILED, tile=512), dict(engine=mc.ENGINE_GRAPH, graph_chunk=7)]):
        net.set_launch(**knobs)
        net.run(250 + 37 * k)
        orc.run(250 + 37 * k)
        assert _same_run(net, orc) > 0


def test_batch_instances_equal_single_runs(conn):
    seeds, scales = [101, 102, 103, 104], [0.02, 0.05, 0.013, 0.03]
    for engine, ring in ((mc.ENGINE_TILED, 0), (mc.ENGINE_TILED, 2), (mc.ENGINE_GRAPH, 0)):
        _say("batch", seeds, scales, "engine", engine, "ring", ring)
        net = mc.Network.build_batch(seeds, scales, conn, engine=engine)
        if ring:
            net.set_launch(engine=mc.ENGINE_TILED, tile=700, ring=ring)
        info = net.info()
        if engine == mc.ENGINE_TILED:
            assert info["n_tiles"] >= 4 and info["lds_ring"] == (0 if ring == 2 else 1)
        net.run(1200)
        for j, (s, sc) in enumerate(zip(seeds, scales)):
            orc = _oracle(s, sc, conn)
            orc.run(1200)
            assert _same_run(net, orc, inst=j) > 0
            assert net.counters(j)["max_spikes_per_step"] == orc.counters()["max_spikes_per_step"]
        tot = net.counters(-1)
        assert tot["spikes"] == sum(net.counters(j)["spikes"] for j in range(4))
        assert tot["max_spikes_per_step"] >= max(net.counters(j)["max_spikes_per_step"] for j in range(4))


def test_global_ring_with_partial_lds_window(conn):
    """Tiles of up to 4096 neurons with the ring in global memory: the LDS left
    over holds only a few of the nearest slots, so events go to both the LDS
    window (short delays) and the global slice (long delays)."""
    seeds, scales = [121, 122], [0.05, 0.05]
    _say("partial lds window")
    net = mc.Network.build_batch(seeds, scales, conn)
    net.set_launch(engine=mc.ENGINE_TILED, tile=4096, ring=2)
    info = net.info()
    assert info["lds_ring"] == 0 and 1 <= info["lds_window"] < 20, info
    for chunk in (700, 500):              # two launches: the window is written back and reloaded
        net.run(chunk)
    for j, (s, sc) in enumerate(zip(seeds, scales)):
        orc = _oracle(s, sc, conn)
        orc.run(1200)
        assert _same_run(net, orc, inst=j) > 0


def test_batch_segments_with_many_spikes(conn):
    """Several 10-15 % instances over 3000 steps: recorder segments of 10^5+
    spikes, drained on the host while the next segment runs, in parallel
    chunks; every instance still equals its single run."""
    seeds, scales = [211, 212, 213, 214, 215, 216], [0.1, 0.12, 0.15, 0.1, 0.11, 0.13]
    _say("batch many spikes", seeds, scales)
    net = mc.Network.build_batch(seeds, scales, conn)
    net.run(3000)
    total = 0
    for j, (s, sc) in enumerate(zip(seeds, scales)):
        orc = _oracle(s, sc, conn)
        orc.run(3000)
        total += _same_run(net, orc, inst=j)
        assert net.counters(j)["events"] == orc.counters()["events"]
        assert net.counters(j)["max_spikes_per_step"] == orc.counters()["max_spikes_per_step"]
    assert total > 100000


@pytest.mark.parametrize("scale", [0.02, 0.1])
def test_dc_workload_parity(conn, scale):
    """The DC-input workload (no Poisson background; each population driven by
    the mean current of its Poisson drive) equals the oracle."""
    from synth_inputs import dc_standin_amplitudes
    _say("dc workload", scale)
    i_dc = dc_standin_amplitudes()
    net = mc.Network.build(9, scale, conn, poisson_on=False, i_dc=i_dc)
    orc = _oracle(9, scale, conn, poisson_on=False, i_dc=i_dc)
    net.run(1500)
    orc.run(1500)
    assert _same_run(net, orc) > 0
    assert net.counters()["poisson_events"] == 0


def test_dc_input_hook_parity(conn):
    _say("dc input")
    i_dc = [420.0, 380.0, 500.0, 0.0, 650.0, 390.0, 0.0, 800.0]
    net = mc.Network.build(6, 0.02, conn, poisson_on=False, i_dc=i_dc)
    orc = _oracle(6, 0.02, conn, poisson_on=False, i_dc=i_dc)
    net.run(2000)
    orc.run(2000)
    assert _same_run(net, orc) > 0


def test_psp_and_state_override(conn):
    """mc_set_state + a single delivered synapse reproduce the oracle's PSP."""
    _say("psp via set_state")
    z = np.zeros(64)
    z[0] = 0.5        # L2/3E -> L2/3E only
    net = mc.Network.build(2, 0.001, z, poisson_on=False, init_mode=1)
    orc = _oracle(2, 0.001, z, poisson_on=False, init_mode=1)
    n, _ = net.size()
    u0 = np.zeros(n, dtype=np.float32)
    u0[0] = 16.0
    net.set_state(u=u0)
    orc.set_state(u=u0.astype(np.float64))
    net.run(60)
    orc.run(60)
    _same_run(net, orc)


def test_edge_cases(conn):
    _say("edge cases")
    net = mc.Network.build(1, 1e-5, conn)             # every population has one neuron
    assert net.info()["engine"] == mc.ENGINE_TILED and net.info()["n_tiles"] == 1
    n, m = net.size()
    assert n == 8
    net.run(0)
    orc = _oracle(1, 1e-5, conn)
    net.run(500)
    orc.run(500)
    _same_run(net, orc)
    with pytest.raises(mc.MCError):
        net.run(-1)
    with pytest.raises(mc.MCError):
        net.state(instance=1)
    tiny = mc.Network.build(1, 0.02, conn, record_capacity=16)
    with pytest.raises(mc.MCError) as e:
        tiny.run(200)
    assert e.value.code == -6


def _check_store_sample(net, orc, rows=64):
    n, m = net.size()
    c_lib = net.csr()
    c_orc = orc.csr()
    assert np.array_equal(c_lib["row_ptr"], c_orc["row_ptr"])
    rng = np.random.default_rng(0)
    for i in rng.choice(n, rows, replace=False):
        a0, a1 = c_lib["row_ptr"][i], c_lib["row_ptr"][i + 1]
        ka = np.lexsort((c_lib["wq"][a0:a1], c_lib["d"][a0:a1], c_lib["post"][a0:a1]))
        kb = np.lexsort((c_orc["wq"][a0:a1], c_orc["d"][a0:a1], c_orc["post"][a0:a1]))
        for f in ("post", "d", "wq"):
            assert np.array_equal(c_lib[f][a0:a1][ka].astype(np.int64), c_orc[f][a0:a1][kb].astype(np.int64))


def test_full_scale_steady_state_parity(conn):
    """Full scale (77,169 neurons, ~3e8 synapses, 256 tiles of 302 neurons):
    sampled rows of the store, then a forced burst -- 3,000 neurons start above
    threshold, so the first step has over 2,048 spikes (several delivery
    batches, ids from entry words) -- and 10^4 steps (1 s) through the
    transient into the steady state, bit-exact.  The delivery-path counters
    show which code paths ran."""
    _say("full scale 10^4 steps, forced burst")
    net = mc.Network.build(1, 1.0, conn)
    info = net.info()
    assert info["engine"] == mc.ENGINE_TILED and info["n_tiles"] == 256 and info["tile_neurons"] == 302
    orc = _oracle(1, 1.0, conn)
    n, m = net.size()
    assert (n, m) == (77169, orc.M)
    assert abs(m / 3e8 - 1) < 0.01
    _check_store_sample(net, orc)
    u, _, _ = orc.state()
    burst = np.random.default_rng(8).choice(n, 3000, replace=False)
    u[burst] = 15.5
    orc.set_state(u=u)
    net.set_state(u=u.astype(np.float32))
    for chunk in (1, 999, 9000):
        net.run(chunk)
        orc.run(chunk)
        assert _same_run(net, orc) > 0
    c, rc = net.counters(), orc.counters()
    for k in ("steps", "spikes", "events", "poisson_events", "max_spikes_per_step"):
        assert c[k] == rc[k], k
    assert c["max_spikes_per_step"] >= 3000
    paths = net.paths()
    _say("delivery paths", paths)
    for k in ("grouped", "per_thread", "extra_batch", "entry_words", "search"):
        assert paths[k] > 0, (k, paths)
    # steady state: most tile-steps take the lane-group path
    assert paths["grouped"] > 0.5 * 256 * 10000


@pytest.mark.parametrize("wfmt", [mc.W_FP16, mc.W_BF16])
def test_full_scale_reduced_precision_parity(conn, wfmt):
    """Full scale with the 4-byte FP16/BF16 records: 2,000 steps bit-exact
    against the oracle's FP16/BF16 mirror."""
    _say("full scale reduced precision", wfmt)
    net = mc.Network.build(1, 1.0, conn, wfmt=wfmt)
    assert net.info()["syn_bytes"] == 4
    orc = _oracle(1, 1.0, conn, wfmt)
    _check_store_sample(net, orc, rows=16)
    for chunk in (500, 1500):
        net.run(chunk)
        orc.run(chunk)
        assert _same_run(net, orc) > 0
    assert net.paths()["grouped"] > 0


@pytest.mark.parametrize("wfmt", [mc.W_FP16, mc.W_BF16])
def test_graph_engine_reduced_precision(conn, wfmt):
    """GRAPH engine with 16-bit weights (the delivery kernel's FP16/BF16 forms)."""
    _say("graph engine reduced precision", wfmt)
    net = mc.Network.build(4, 0.02, conn, wfmt=wfmt, engine=mc.ENGINE_GRAPH)
    assert net.info()["engine"] == mc.ENGINE_GRAPH and net.info()["syn_bytes"] == 7
    orc = _oracle(4, 0.02, conn, wfmt)
    net.run(3000)
    orc.run(3000)
    assert _same_run(net, orc) > 100


@pytest.mark.parametrize("wfmt", [mc.W_FP16, mc.W_BF16])
def test_eight_byte_reduced_precision_records(conn, wfmt):
    """Tiles over 1,024 neurons: FP16/BF16 weights in 8-byte records (two
    neurons per thread, ring in global memory)."""
    _say("8-byte 16-bit records", wfmt)
    net = mc.Network.build(12, 0.05, conn, wfmt=wfmt)
    net.set_launch(engine=mc.ENGINE_TILED, tile=2000, ring=2)
    info = net.info()
    assert info["syn_bytes"] == 8 and info["tile_neurons"] > 1024
    orc = _oracle(12, 0.05, conn, wfmt)
    net.run(1500)
    orc.run(1500)
    assert _same_run(net, orc) > 100


@pytest.mark.parametrize("budget", [0.0, 1e6])
def test_trace_form_parity(conn, budget):
    """The phase-trace form of the step kernel (alone, and with an ample step
    budget: the trace and budget form) gives the same results."""
    _say("trace form, budget", budget)
    net = mc.Network.build(13, 0.2, conn)
    orc = _oracle(13, 0.2, conn)
    if budget:
        net.set_step_budget(budget)
    net.set_trace(400)
    net.run(700)
    orc.run(700)
    assert _same_run(net, orc) > 100
    tr = net.trace()
    assert tr.shape == (400, net.info()["n_tiles"], 8)
    assert np.all(tr[1:, :, 0] > tr[:-1, :, 0])          # step start times increase
    assert net.counters()["dropped_events"] == 0


def test_ordinary_launch_parity(conn):
    """The tiled kernel started by an ordinary (not cooperative) launch."""
    _say("ordinary launch")
    net = mc.Network.build(14, 0.1, conn)
    net.set_launch(coop=2)
    orc = _oracle(14, 0.1, conn)
    for chunk in (20, 980):
        net.run(chunk)
        orc.run(chunk)
        assert _same_run(net, orc) > 0


@pytest.mark.parametrize("scale,steps", [(0.02, 2000), (1.0, 500)])
def test_relaxed_start_parity(conn, scale, steps):
    """The relaxed initial state (init_mode 2: per-population moments of u and
    I from the stand-in's steady state) drawn by the library equals the
    oracle's, and the run from it too."""
    from synth_inputs import relaxed_start
    _say("relaxed start", scale)
    kw = relaxed_start()
    net = mc.Network.build(5, scale, conn, **kw)
    orc = _oracle(5, scale, conn, **kw)
    u, I, r = net.state()
    ru, rI, rr = orc.state()
    assert np.array_equal(u.astype(np.float64), ru) and np.array_equal(I.astype(np.float64), rI)
    assert u.max() < 15.0 and I.std() > 0
    net.run(steps)
    orc.run(steps)
    assert _same_run(net, orc) > 0


def test_checkpoint_resume_is_bit_exact(conn, tmp_path):
    _say("checkpoint")
    path = str(tmp_path / "net.ckpt")
    a = mc.Network.build(41, 0.05, conn)
    a.run(500)
    a.spikes()
    a.save(path)
    a.run(700)
    sa = a.spikes()
    ua = a.state()
    b = mc.Network.build(41, 0.05, conn, engine=mc.ENGINE_GRAPH)     # resume on the other engine
    b.load(path)
    b.run(700)
    sb = b.spikes()
    assert len(sa[0]) > 0
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    for x, y in zip(ua, b.state()):
        assert np.array_equal(x, y)
    assert a.counters() == b.counters()
    other = mc.Network.build(42, 0.05, conn)
    with pytest.raises(mc.MCError) as e:
        other.load(path)
    assert e.value.code == -1


def test_event_counts_with_undrained_spikes(conn, tmp_path):
    """A short record's event counts (sums of the spiking neurons' out-degrees)
    are taken when they are read: counters read while spikes are still waiting
    to be drained, after a checkpoint saved with spikes waiting, and per
    instance of a batch all equal the oracle's."""
    _say("event counts with undrained spikes")
    path = str(tmp_path / "pending.ckpt")
    net = mc.Network.build(43, 0.05, conn)
    orc = _oracle(43, 0.05, conn)
    keys = ("steps", "spikes", "events", "max_spikes_per_step")
    for steps in (7, 40, 300):
        net.run(steps)
        orc.run(steps)
        c, rc = net.counters(), orc.counters()
        assert all(c[k] == rc[k] for k in keys), (c, rc)
    assert c["events"] > 0
    net.save(path)                      # spikes of 347 steps still undrained
    other = mc.Network.build(43, 0.05, conn)
    other.load(path)
    assert other.counters() == net.counters()
    st, ids = other.spikes()
    assert len(st) == c["spikes"]
    assert _same_run(net, orc) == c["spikes"]
    net.run(200)
    orc.run(200)
    c, rc = net.counters(), orc.counters()
    assert all(c[k] == rc[k] for k in keys), (c, rc)
    # per instance: instance 1 of a batch against its own oracle
    batch = mc.Network.build_batch([43, 44], [0.05, 0.02], conn)
    o1 = _oracle(44, 0.02, conn)
    batch.run(250)
    o1.run(250)
    c1, r1 = batch.counters(1), o1.counters()
    assert c1["spikes"] == r1["spikes"] and c1["events"] == r1["events"]
    assert batch.counters()["events"] == c1["events"] + batch.counters(0)["events"]


def test_rewind_then_new_dynamics(conn, tmp_path):
    """Loading a checkpoint moves the step index back; the spike-exchange words
    written for the abandoned steps carry the tags the resumed run polls for and
    must not be taken for its own (here the resumed run differs: u is halved)."""
    _say("rewind")
    path = str(tmp_path / "rw.ckpt")
    net = mc.Network.build(44, 0.2, conn)
    orc = _oracle(44, 0.2, conn)
    net.run(300)
    orc.run(300)
    assert _same_run(net, orc) > 0
    net.save(path)
    net.run(600)                      # the abandoned future
    net.spikes()
    net.load(path)
    u, I, r = orc.state()
    u2 = (u.astype(np.float32) * np.float32(0.5)).astype(np.float64)
    net.set_state(u=u2.astype(np.float32))
    orc.set_state(u=u2)
    net.run(600)
    orc.run(600)
    assert _same_run(net, orc) > 0


def test_step_budget_off_or_ample_changes_nothing(conn):
    """Lossy real-time mode: a budget no step comes near delivers everything,
    exactly as without one."""
    _say("step budget ample")
    net = mc.Network.build(45, 0.05, conn)
    orc = _oracle(45, 0.05, conn)
    net.set_step_budget(1e6)
    net.run(1500)
    orc.run(1500)
    assert _same_run(net, orc) > 0
    assert net.counters()["dropped_events"] == 0


def test_step_budget_spent_drops_every_event(conn):
    """With a budget of one clock tick every tile finds it spent before its first
    delivery round, so every recurrent event is dropped and counted: the run
    equals the oracle's run of the same neurons without synapses, and the
    dropped count equals the events of the recorded spikes."""
    _say("step budget spent")
    net = mc.Network.build(46, 0.05, conn)
    orc = _oracle(46, 0.05, np.zeros(64))
    net.set_step_budget(0.01)
    net.run(1500)
    orc.run(1500)
    assert _same_run(net, orc) > 0
    c = net.counters()
    assert c["events"] > 0 and c["dropped_events"] == c["events"]
    net.set_step_budget(0)
    with pytest.raises(mc.MCError):
        net.set_step_budget(-1)
    g = mc.Network.build(46, 0.05, conn, engine=mc.ENGINE_GRAPH)
    g.set_step_budget(5.0)
    with pytest.raises(mc.MCError) as e:
        g.run(10)
    assert e.value.code == -9          # MC_ERR_UNSUPPORTED


def test_autotuner_keeps_results(conn):
    _say("autotune")
    net = mc.Network.build(43, 0.05, conn)
    orc = _oracle(43, 0.05, conn)
    net.run(300)
    orc.run(300)
    net.tune(200)                     # trials run on a copy of the state and are rolled back
    assert net.counters()["steps"] == 300
    net.run(900)
    orc.run(900)
    assert _same_run(net, orc) > 0


def test_full_scale_global_ring_variant(conn):
    """Full scale with the tile rings in global memory (owner-computes)."""
    _say("full scale global ring")
    net = mc.Network.build(2, 1.0, conn)
    net.set_launch(engine=mc.ENGINE_TILED, ring=2)
    assert net.info()["lds_ring"] == 0
    orc = _oracle(2, 1.0, conn)
    net.run(90)
    orc.run(90)
    assert _same_run(net, orc) > 0


@pytest.mark.parametrize("wfmt,lanes", [(mc.W_FP32, 3), (mc.W_FP32, 16), (mc.W_FP16, 0), (mc.W_BF16, 5)])
def test_injection_record_forms(conn, wfmt, lanes):
    """Injection reads the store in aligned 16-byte chunks (two 8-byte or four
    4-byte records) and masks the records of neighbouring sub-rows at both ends:
    every record form, and lane counts that leave a ragged last group, give the
    oracle's ring, bit for bit."""
    _say("injection record forms", wfmt, lanes)
    net = mc.Network.build(52, 0.1, conn, wfmt=wfmt)
    if lanes:
        net.set_launch(lanes=lanes)
    orc = _oracle(52, 0.1, conn, wfmt)
    rng = np.random.default_rng(6)
    n = net.size()[0]
    for k in range(2):
        ids = rng.integers(0, n, 3000 if k == 0 else 9000)   # the second list spans two batches
        ev = net.inject_spikes(ids)
        orc.inject(ids)
        assert ev == int(np.diff(orc.csr()["row_ptr"])[ids].sum())
        net.run(60)
        orc.run(60)
        assert _same_run(net, orc) > 0


def test_full_scale_injection_parity(conn):
    """Full scale, the delivery benchmark's shape: 20,000 listed neurons
    delivered at once into the 256 tiles' rings, then 30 steps bit-exact.  The
    injected input is net inhibitory and silences the network for these steps,
    so the check is the state: every neuron's synaptic current and membrane
    potential, which the injected events decide, equal to the oracle's."""
    _say("full scale injection")
    net = mc.Network.build(3, 1.0, conn)
    orc = _oracle(3, 1.0, conn)
    ids = np.random.default_rng(9).choice(net.size()[0], 20000, replace=False)
    ev = net.inject_spikes(ids)
    orc.inject(ids)
    assert ev == int(np.diff(orc.csr()["row_ptr"])[ids].sum()) > 7e7
    net.run(30)
    orc.run(30)
    _same_run(net, orc)
    _, I, _ = orc.state()
    assert np.count_nonzero(I) > 0.99 * len(I)


@pytest.mark.parametrize("engine", [mc.ENGINE_TILED, mc.ENGINE_GRAPH])
def test_injected_spikes_parity(conn, engine):
    """External stimulation: rows of chosen neurons delivered as if they spiked."""
    _say("inject", engine)
    net = mc.Network.build(51, 0.05, conn, engine=engine)
    orc = _oracle(51, 0.05, conn)
    rng = np.random.default_rng(5)
    for k in range(3):
        ids = rng.integers(0, net.size()[0], 40 + 500 * k)      # repeats allowed
        ev = net.inject_spikes(ids)
        orc.inject(ids)
        c = orc.csr()
        assert ev == int(np.diff(c["row_ptr"])[ids].sum())
        net.run(150)
        orc.run(150)
        assert _same_run(net, orc) > 0
    with pytest.raises(mc.MCError):
        net.inject_spikes([net.size()[0]])
