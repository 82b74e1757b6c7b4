"""ctypes binding of libmc (argument marshalling only; every step of the
simulation runs in the library's HIP kernels)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmc.so")

MC_OK = 0
ERRORS = {-1: "MC_ERR_ARG", -2: "MC_ERR_NOMEM", -3: "MC_ERR_HIP", -4: "MC_ERR_OVERFLOW_BOUND",
          -5: "MC_ERR_DELAY_RANGE", -6: "MC_ERR_RECORD_OVERFLOW", -7: "MC_ERR_BUFFER_TOO_SMALL",
          -8: "MC_ERR_IO", -9: "MC_ERR_UNSUPPORTED"}
W_FP32, W_FP16, W_BF16 = 0, 1, 2
ENGINE_AUTO, ENGINE_GRAPH, ENGINE_TILED = 0, 1, 2
NPOP = 8


class MCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class McConfig(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("conn_probs", C.POINTER(C.c_double)),
        ("wfmt", C.c_int32), ("poisson_on", C.c_int32), ("init_mode", C.c_int32), ("engine", C.c_int32),
        ("record_capacity", C.c_int64),
        ("full_size", C.c_double * NPOP), ("k_ext", C.c_double * NPOP), ("i_dc_pa", C.c_double * NPOP),
        ("nu_bg_hz", C.c_double), ("dt_ms", C.c_double), ("tau_m_ms", C.c_double), ("c_m_pf", C.c_double),
        ("tau_syn_ms", C.c_double), ("t_ref_ms", C.c_double), ("theta_mv", C.c_double),
        ("w_mean_pa", C.c_double), ("w_sd_pa", C.c_double), ("g", C.c_double),
        ("l4e_l23e_factor", C.c_double), ("w_ext_pa", C.c_double),
        ("d_mean_exc_ms", C.c_double), ("d_sd_exc_ms", C.c_double),
        ("d_mean_inh_ms", C.c_double), ("d_sd_inh_ms", C.c_double),
        ("device_build", C.c_int32),
        ("init_u_mean_mv", C.c_double * NPOP), ("init_u_sd_mv", C.c_double * NPOP),
        ("init_i_mean_pa", C.c_double * NPOP), ("init_i_sd_pa", C.c_double * NPOP),
    ]


class McCounters(C.Structure):
    _fields_ = [("steps", C.c_int64), ("spikes", C.c_int64), ("events", C.c_int64),
                ("poisson_events", C.c_int64), ("max_spikes_per_step", C.c_int64), ("dropped_events", C.c_int64)]


class McInfo(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("ring_depth", C.c_int32), ("engine", C.c_int32), ("wfmt", C.c_int32),
                ("n_neurons", C.c_int64), ("n_synapses", C.c_int64), ("tile_neurons", C.c_int32),
                ("n_tiles", C.c_int32), ("graph_chunk", C.c_int32), ("seg", C.c_int32), ("block", C.c_int32),
                ("deliver_grid", C.c_int32), ("lds_ring", C.c_int32), ("syn_bytes", C.c_int32),
                ("poll_delay", C.c_int32), ("lds_window", C.c_int32)]


class McLaunch(C.Structure):
    _fields_ = [("engine", C.c_int32), ("tile", C.c_int32), ("ring", C.c_int32), ("graph_chunk", C.c_int32), ("seg", C.c_int32), ("block", C.c_int32),
                ("deliver_grid", C.c_int32), ("poll_delay", C.c_int32), ("coop", C.c_int32), ("lanes", C.c_int32)]


# Every entry point declared in include/mc.h.
EXPORTS = ("mc_config_default", "mc_build_network", "mc_build_batch", "mc_run", "mc_get_spikes",
           "mc_get_state", "mc_set_state", "mc_get_counters", "mc_get_info", "mc_get_csr",
           "mc_instance_size", "mc_set_launch", "mc_tune", "mc_set_stream", "mc_set_timing",
           "mc_get_timing", "mc_set_trace", "mc_get_trace", "mc_save_state", "mc_load_state", "mc_free",
           "mc_last_error", "mc_inject_spikes", "mc_set_step_budget", "mc_set_wait_limit",
           "mc_get_paths", "mc_probe", "mc_inject_spikes_noalloc")

_lib = None


def lib():
    """Load libmc.so.  There is no fallback: without the built HIP library the
    simulator does not run."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmc.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_1909_08665_amd.build`")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # soname); loading torch first makes libmc bind to that copy instead of
    # mapping a second runtime next to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    L.mc_last_error.restype = C.c_char_p
    L.mc_config_default.argtypes = [C.POINTER(McConfig)]
    L.mc_build_network.argtypes = [C.c_uint64, C.c_double, C.POINTER(McConfig), C.POINTER(P)]
    L.mc_build_batch.argtypes = [P, P, I32, C.POINTER(McConfig), C.POINTER(P)]
    L.mc_run.argtypes = [P, I64]
    L.mc_get_spikes.argtypes = [P, I32, P, P, I64, C.POINTER(I64)]
    L.mc_get_state.argtypes = [P, I32, P, P, P, I64]
    L.mc_set_state.argtypes = [P, I32, P, P, P, I64]
    L.mc_get_counters.argtypes = [P, I32, C.POINTER(McCounters)]
    L.mc_get_info.argtypes = [P, C.POINTER(McInfo)]
    L.mc_get_csr.argtypes = [P, I32, P, P, P, P, I64]
    L.mc_instance_size.argtypes = [P, I32, C.POINTER(I64), C.POINTER(I64)]
    L.mc_set_launch.argtypes = [P, C.POINTER(McLaunch)]
    L.mc_tune.argtypes = [P, I64]
    L.mc_set_stream.argtypes = [P, P]
    L.mc_set_timing.argtypes = [P, I32]
    L.mc_get_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(I64)]
    L.mc_inject_spikes.argtypes = [P, I32, P, I64, C.POINTER(I64)]
    L.mc_inject_spikes_noalloc.argtypes = [P, I32, P, I64, C.POINTER(I64)]
    L.mc_set_trace.argtypes = [P, I32]
    L.mc_get_trace.argtypes = [P, P, I64, C.POINTER(I64)]
    L.mc_save_state.argtypes = [P, C.c_char_p]
    L.mc_load_state.argtypes = [P, C.c_char_p]
    L.mc_set_step_budget.argtypes = [P, C.c_double]
    L.mc_set_wait_limit.argtypes = [P, I64]
    L.mc_get_paths.argtypes = [P, P, I32]
    L.mc_probe.argtypes = [I32, I64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.mc_free.argtypes = [P]
    L.mc_free.restype = None
    _lib = L
    return L


PROBE_HBM_COPY, PROBE_LDS_ATOMICS, PROBE_DEVICE_ATOMICS, PROBE_HBM_GATHER = 0, 1, 2, 3


def probe(kind, nbytes=0):
    """Memory-system ceiling on the current device: (rate, kernel ms); rate in
    GB/s for PROBE_HBM_COPY and PROBE_HBM_GATHER, atomics/s for the atomic probes."""
    rate, ms = C.c_double(), C.c_double()
    _check(lib().mc_probe(int(kind), int(nbytes), C.byref(rate), C.byref(ms)))
    return rate.value, ms.value


def _check(rc):
    if rc != MC_OK:
        raise MCError(rc, lib().mc_last_error().decode())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_config(conn, *, wfmt=W_FP32, poisson_on=True, init_mode=0, engine=ENGINE_AUTO,
                record_capacity=0, i_dc=None, **params):
    """mc_config with the library defaults, the given table and overrides."""
    cfg = McConfig()
    _check(lib().mc_config_default(C.byref(cfg)))
    conn = np.ascontiguousarray(np.asarray(conn, dtype=np.float64).reshape(64))
    cfg.conn_probs = conn.ctypes.data_as(C.POINTER(C.c_double))
    cfg._keep = conn          # keep the table alive as long as the config
    cfg.wfmt, cfg.poisson_on, cfg.init_mode, cfg.engine = wfmt, int(bool(poisson_on)), init_mode, engine
    cfg.record_capacity = record_capacity
    if i_dc is not None:
        cfg.i_dc_pa[:] = [float(x) for x in i_dc]
    for k, v in params.items():
        if k in ("full_size", "k_ext", "init_u_mean_mv", "init_u_sd_mv", "init_i_mean_pa", "init_i_sd_pa"):
            getattr(cfg, k)[:] = [float(x) for x in v]
        else:
            setattr(cfg, k, v)
    return cfg


class Network:
    """A microcircuit (or a batch of independent instances) resident on the GPU."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    @classmethod
    def build(cls, seed, scale, conn, **cfg_kw):
        cfg = make_config(conn, **cfg_kw)
        h = C.c_void_p()
        _check(lib().mc_build_network(C.c_uint64(int(seed)), float(scale), C.byref(cfg), C.byref(h)))
        return cls(h.value)

    @classmethod
    def build_batch(cls, seeds, scales, conn, **cfg_kw):
        cfg = make_config(conn, **cfg_kw)
        s = np.ascontiguousarray(seeds, dtype=np.uint64)
        sc = np.ascontiguousarray(scales, dtype=np.float64)
        if len(s) != len(sc):
            raise ValueError("seeds and scales differ in length")
        h = C.c_void_p()
        _check(lib().mc_build_batch(_ptr(s), _ptr(sc), len(s), C.byref(cfg), C.byref(h)))
        return cls(h.value)

    def close(self):
        if self._h is not None and self._h.value:
            lib().mc_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- running -----------------------------------------------------------
    def run(self, steps):
        _check(lib().mc_run(self._h, int(steps)))

    def set_launch(self, engine=0, tile=0, ring=0, graph_chunk=0, seg=0, block=0, deliver_grid=0, poll_delay=0,
                   coop=0, lanes=0):
        """ring: 0 auto, 1 tile ring in LDS, 2 tile ring in global memory (tiled engine).
        poll_delay: tiled engine, sleep before polling in units of 64 clocks (-1 none).
        coop: tiled engine, 1 cooperative launch, 2 ordinary launch.
        lanes: tiled engine, lanes per spike for cursor delivery (1..64).
        0 keeps the current value of any knob."""
        l = McLaunch(engine, tile, ring, graph_chunk, seg, block, deliver_grid, poll_delay, coop, lanes)
        _check(lib().mc_set_launch(self._h, C.byref(l)))

    def set_step_budget(self, budget_us):
        """Lossy real-time mode (tiled engine): per step, events not delivered
        within budget_us of the step's start are dropped and counted in
        counters()["dropped_events"]; 0 turns it off."""
        _check(lib().mc_set_step_budget(self._h, float(budget_us)))

    def set_wait_limit(self, polls):
        """Polls after which a cross-tile wait of the tiled engine gives up
        (0: at once, to exercise the failure path)."""
        _check(lib().mc_set_wait_limit(self._h, int(polls)))

    PATHS = ("no_spikes", "grouped", "fast", "per_thread", "batched", "extra_batch", "direct_map", "search",
             "entry_words")

    def paths(self):
        """Tile-steps per delivery path of the tiled engine (coverage counters)."""
        out = np.zeros(len(self.PATHS), dtype=np.int64)
        _check(lib().mc_get_paths(self._h, _ptr(out), len(out)))
        return dict(zip(self.PATHS, out.tolist()))

    def tune(self, trial_steps=200):
        _check(lib().mc_tune(self._h, int(trial_steps)))

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream (HIP stream) or None for the library's own."""
        handle = None if stream is None else C.c_void_p(stream.cuda_stream)
        _check(lib().mc_set_stream(self._h, handle))

    def set_timing(self, on=True):
        _check(lib().mc_set_timing(self._h, int(bool(on))))

    def timing(self):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().mc_get_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def inject_spikes(self, ids, instance=0):
        """Deliver the rows of neurons `ids` as if they spiked in the last step;
        returns the number of synapses delivered."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        ev = C.c_int64()
        _check(lib().mc_inject_spikes(self._h, int(instance), _ptr(ids), len(ids), C.byref(ev)))
        return ev.value

    def inject_spikes_noalloc(self, ids, instance=0):
        """inject_spikes with the ids staged in the library's fixed per-GPU
        array (no device allocation; at most 2^20 ids)."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        ev = C.c_int64()
        _check(lib().mc_inject_spikes_noalloc(self._h, int(instance), _ptr(ids), len(ids), C.byref(ev)))
        return ev.value

    def set_trace(self, steps):
        """Record per-step phase timestamps for the first `steps` steps of the next run."""
        _check(lib().mc_set_trace(self._h, int(steps)))

    def trace(self, launch=False):
        """[steps, tiles, 8] uint64: 100 MHz timestamps of the step phases (slot 7:
        the step's spike count); with launch=True also the [tiles, 4] launch
        timestamps (entry, first step, end of the last step, end of write-back)."""
        cnt = C.c_int64()
        lib().mc_get_trace(self._h, None, 0, C.byref(cnt))
        out = np.zeros(cnt.value, dtype=np.uint64)
        if cnt.value:
            _check(lib().mc_get_trace(self._h, _ptr(out), cnt.value, C.byref(cnt)))
        info = self.info()
        rows = out.reshape(-1, max(1, info["n_tiles"]), 8)
        steps = rows[:-1] if len(rows) else rows
        return (steps, rows[-1, :, :7] if len(rows) else None) if launch else steps

    def save(self, path):
        _check(lib().mc_save_state(self._h, os.fsencode(path)))

    def load(self, path):
        _check(lib().mc_load_state(self._h, os.fsencode(path)))

    # -- inspection ------------------------------------------------------------
    def size(self, instance=0):
        n, m = C.c_int64(), C.c_int64()
        _check(lib().mc_instance_size(self._h, int(instance), C.byref(n), C.byref(m)))
        return n.value, m.value

    def info(self):
        i = McInfo()
        _check(lib().mc_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in McInfo._fields_}

    def spikes(self, instance=0):
        """(steps, ids) recorded since the last call, sorted by (step, id)."""
        cnt = C.c_int64()
        rc = lib().mc_get_spikes(self._h, int(instance), None, None, 0, C.byref(cnt))
        if rc not in (MC_OK, -7):
            _check(rc)
        steps = np.zeros(cnt.value, dtype=np.int64)
        ids = np.zeros(cnt.value, dtype=np.int32)
        _check(lib().mc_get_spikes(self._h, int(instance), _ptr(steps), _ptr(ids), cnt.value, C.byref(cnt)))
        return steps[:cnt.value], ids[:cnt.value]

    def state(self, instance=0):
        n, _ = self.size(instance)
        u = np.zeros(n, dtype=np.float32)
        I = np.zeros(n, dtype=np.float32)
        r = np.zeros(n, dtype=np.int32)
        _check(lib().mc_get_state(self._h, int(instance), _ptr(u), _ptr(I), _ptr(r), n))
        return u, I, r

    def set_state(self, instance=0, u=None, I=None, refr=None):
        n, _ = self.size(instance)
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float32)
        I = None if I is None else np.ascontiguousarray(I, dtype=np.float32)
        refr = None if refr is None else np.ascontiguousarray(refr, dtype=np.int32)
        _check(lib().mc_set_state(self._h, int(instance), _ptr(u), _ptr(I), _ptr(refr), n))

    def counters(self, instance=-1):
        c = McCounters()
        _check(lib().mc_get_counters(self._h, int(instance), C.byref(c)))
        return {f: getattr(c, f) for f, _ in McCounters._fields_}

    def csr(self, instance=0):
        n, m = self.size(instance)
        rp = np.zeros(n + 1, dtype=np.int64)
        post = np.zeros(m, dtype=np.int32)
        wq = np.zeros(m, dtype=np.int32)
        d = np.zeros(m, dtype=np.uint8)
        _check(lib().mc_get_csr(self._h, int(instance), _ptr(rp), _ptr(post), _ptr(wq), _ptr(d), m))
        return dict(row_ptr=rp, post=post, wq=wq, d=d)
