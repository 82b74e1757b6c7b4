"""mc_inject_spikes_noalloc: the injection entry point that allocates nothing
(ids staged in the library's fixed per-GPU array) gives exactly what
mc_inject_spikes gives, on two calls in a row (the second with fewer ids),
and refuses a list longer than its array."""
import numpy as np
import pytest

import paper_1909_08665_amd as mc
from synth_inputs import standin_conn_table

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("engine", [mc.ENGINE_TILED, mc.ENGINE_GRAPH])
def test_noalloc_injection_equals_allocating_one(engine):
    print(f"[case] no-alloc injection, engine {engine}", flush=True)
    conn = standin_conn_table()
    a = mc.Network.build(81, 0.05, conn, engine=engine)
    b = mc.Network.build(81, 0.05, conn, engine=engine)
    n, _ = a.size()
    rng = np.random.default_rng(9)
    for k, count in enumerate((3000, 700)):                 # the second call smaller
        ids = rng.integers(0, n, count)
        ea = a.inject_spikes(ids)
        eb = b.inject_spikes_noalloc(ids)
        assert ea == eb > 0
        a.run(120 + 30 * k)
        b.run(120 + 30 * k)
        sa, sb = a.spikes(), b.spikes()
        assert len(sa[0]) > 0
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
        for x, y in zip(a.state(), b.state()):
            assert np.array_equal(x, y)
    with pytest.raises(mc.MCError) as e:
        b.inject_spikes_noalloc(np.zeros((1 << 20) + 1, dtype=np.int32))
    assert e.value.code == -1
    with pytest.raises(mc.MCError):
        b.inject_spikes_noalloc([n])
