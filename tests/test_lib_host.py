"""Host-side checks of libmc: the library loads, exports every entry point that
include/mc.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1909_08665_amd as mc
from paper_1909_08665_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(mc_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    assert sorted(mc.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = mc.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_config_defaults():
    cfg = B.McConfig()
    assert mc.lib().mc_config_default(C.byref(cfg)) == 0
    assert cfg.struct_size == C.sizeof(B.McConfig)
    assert (cfg.dt_ms, cfg.tau_m_ms, cfg.c_m_pf, cfg.tau_syn_ms, cfg.t_ref_ms, cfg.theta_mv) == (0.1, 10.0, 250.0, 0.5, 2.0, 15.0)
    assert (cfg.w_mean_pa, cfg.w_sd_pa, cfg.g, cfg.w_ext_pa) == (87.8, 8.78, -4.0, 87.8)
    assert list(cfg.full_size) == [20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948]
    assert list(cfg.k_ext) == [1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100]
    assert not cfg.conn_probs


def test_missing_table_and_bad_args_rejected():
    L = mc.lib()
    h = C.c_void_p()
    assert L.mc_build_network(1, 0.02, None, C.byref(h)) == -1
    assert b"conn" in L.mc_last_error()
    cfg = B.McConfig()
    L.mc_config_default(C.byref(cfg))
    assert L.mc_build_network(1, 0.02, C.byref(cfg), C.byref(h)) == -1     # conn_probs NULL
    conn = np.full(64, 0.05)
    for bad_conn in (np.full(64, 1.0), np.full(64, -0.1)):
        with pytest.raises(mc.MCError) as e:
            mc.Network.build(1, 0.02, bad_conn)
        assert e.value.code == -1
    with pytest.raises(mc.MCError):
        mc.Network.build(1, 0.0, conn)
    with pytest.raises(mc.MCError):
        mc.Network.build(1, 1.5, conn)
    with pytest.raises(mc.MCError):
        mc.Network.build(1, 0.02, conn, wfmt=7)
    with pytest.raises(mc.MCError):
        mc.Network.build(1, 0.02, conn, tau_syn_ms=10.0)
    with pytest.raises(mc.MCError):
        mc.Network.build(1, 0.02, conn, device_build=2)
    assert L.mc_run(None, 1) == -1
    assert L.mc_set_step_budget(None, 5.0) == -1
    assert L.mc_set_launch(None, None) == -1
    assert L.mc_inject_spikes(None, 0, None, 0, None) == -1
    # probes: unknown kind, buffer size out of range, no result pointer
    rate, ms = C.c_double(), C.c_double()
    assert L.mc_probe(4, 1 << 20, C.byref(rate), C.byref(ms)) == -1
    assert L.mc_probe(-1, 1 << 20, C.byref(rate), C.byref(ms)) == -1
    assert L.mc_probe(mc.PROBE_HBM_GATHER, 4096, C.byref(rate), C.byref(ms)) == -1
    assert L.mc_probe(mc.PROBE_HBM_COPY, 1 << 37, C.byref(rate), C.byref(ms)) == -1
    assert L.mc_probe(mc.PROBE_HBM_COPY, 1 << 20, None, None) == -1
    L.mc_free(None)


def test_overflow_bound_refused_before_upload(conn_table):
    """Absurd weights: the host builder refuses the network with
    MC_ERR_OVERFLOW_BOUND (int32 input buffers) before any device memory is
    touched, as the oracle does for the same parameters."""
    with pytest.raises(mc.MCError) as e:
        mc.Network.build(1, 0.1, conn_table, w_mean_pa=1.5e4, w_sd_pa=10.0)
    assert e.value.code == -4
    assert b"overflow" in mc.lib().mc_last_error()


def _no_gpu():
    try:
        import torch
        return torch.cuda.device_count() == 0
    except Exception:
        return True


@pytest.mark.skipif(not _no_gpu(), reason="only meaningful on a machine without a GPU")
def test_fails_loudly_without_gpu(conn_table):
    with pytest.raises(mc.MCError) as e:
        mc.Network.build(1, 0.02, conn_table)
    assert e.value.code in (-2, -3)
