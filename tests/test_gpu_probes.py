"""The memory-system probes behind the roofline figures: each returns a
positive rate within what the device can physically do, and the LDS atomic
probe checks that every add landed (it fails otherwise)."""
import pytest

import paper_1909_08665_amd as mc

pytestmark = pytest.mark.gpu

HBM_PEAK_GBS = 8000.0


def _say(*a):
    print("[case]", *a, flush=True)


def test_streaming_copy_and_gather_rates():
    _say("probe copy + gather")
    copy, ms = mc.probe(mc.PROBE_HBM_COPY, 1 << 30)
    assert ms > 0 and 500.0 < copy < 1.05 * HBM_PEAK_GBS, copy
    gather, ms = mc.probe(mc.PROBE_HBM_GATHER, 1 << 30)
    assert ms > 0 and 100.0 < gather < 1.05 * HBM_PEAK_GBS, gather
    # a buffer that fits the caches reads faster than one spread over HBM
    small, _ = mc.probe(mc.PROBE_HBM_GATHER, 1 << 20)
    assert small > gather, (small, gather)


def test_atomic_rates():
    _say("probe atomics")
    lds, ms = mc.probe(mc.PROBE_LDS_ATOMICS)
    assert ms > 0 and lds > 1e11, lds
    dev, ms = mc.probe(mc.PROBE_DEVICE_ATOMICS, 1 << 20)
    assert ms > 0 and 1e9 < dev < lds, (dev, lds)
