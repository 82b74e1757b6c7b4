"""CPU oracle for the cortical-microcircuit simulation -- Python wrapper.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use this module; the simulator library never imports it and shares
no code with it.

The arithmetic lives in ``mc_oracle.c`` (plain C, one obvious loop per model
step); this file holds the oracle's own copy of the model constants (Sec. 2a of
Rhodes et al., arXiv 1909.08665, and the microcircuit workload sizes) and a thin
ctypes wrapper.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mc_oracle.c")
LIB = os.path.join(HERE, "libmc_oracle.so")

NPOP = 8
KMAX = 24
POP_NAMES = ("L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I")
# Full-scale population sizes and background in-degrees of the microcircuit
# workload (77,169 neurons; 8 Hz Poisson sources).
FULL_SIZE = (20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948)
K_EXT = (1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100)

MIRROR, FP64 = 0, 1
W_FP32, W_FP16, W_BF16 = 0, 1, 2


class OrParams(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("wfmt", C.c_int32), ("poisson_on", C.c_int32), ("init_mode", C.c_int32),
        ("full_size", C.c_double * NPOP), ("k_ext", C.c_double * NPOP), ("i_dc_pa", C.c_double * NPOP),
        ("nu_bg_hz", C.c_double), ("dt_ms", C.c_double),
        ("tau_m_ms", C.c_double), ("c_m_pf", C.c_double), ("tau_syn_ms", C.c_double),
        ("t_ref_ms", C.c_double), ("theta_mv", C.c_double),
        ("w_mean_pa", C.c_double), ("w_sd_pa", C.c_double), ("g", C.c_double),
        ("l4e_l23e_factor", C.c_double), ("w_ext_pa", C.c_double),
        ("d_mean_exc_ms", C.c_double), ("d_sd_exc_ms", C.c_double),
        ("d_mean_inh_ms", C.c_double), ("d_sd_inh_ms", C.c_double),
        ("pois_stream", C.c_uint64),
        ("init_u_mean_mv", C.c_double * NPOP), ("init_u_sd_mv", C.c_double * NPOP),
        ("init_i_mean_pa", C.c_double * NPOP), ("init_i_sd_pa", C.c_double * NPOP),
    ]


def default_params(mode=MIRROR, wfmt=W_FP32, poisson_on=True, init_mode=0, i_dc=None, **over):
    """Model constants of Sec. 2a (with the workload's delay values)."""
    p = OrParams()
    p.mode, p.wfmt, p.poisson_on, p.init_mode = mode, wfmt, int(bool(poisson_on)), init_mode
    p.full_size[:] = [float(x) for x in FULL_SIZE]
    p.k_ext[:] = [float(x) for x in K_EXT]
    p.i_dc_pa[:] = [0.0] * NPOP if i_dc is None else [float(x) for x in i_dc]
    p.nu_bg_hz, p.dt_ms = 8.0, 0.1
    p.tau_m_ms, p.c_m_pf, p.tau_syn_ms, p.t_ref_ms = 10.0, 250.0, 0.5, 2.0
    p.theta_mv = 15.0          # V_th - E_L = -50 - (-65) mV
    p.w_mean_pa, p.w_sd_pa, p.g, p.l4e_l23e_factor = 87.8, 8.78, -4.0, 2.0
    p.w_ext_pa = 87.8
    p.d_mean_exc_ms, p.d_sd_exc_ms, p.d_mean_inh_ms, p.d_sd_inh_ms = 1.5, 0.75, 0.8, 0.4
    p.pois_stream = 0
    for k, v in over.items():
        if k.startswith("init_") and k != "init_mode":
            getattr(p, k)[:] = [float(x) for x in v]
        else:
            setattr(p, k, v)
    return p


def build_library(force=False):
    """Compile the oracle with gcc (no contraction, IEEE semantics)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = build_library()
    L = C.CDLL(path)
    P = C.c_void_p
    L.or_last_error.restype = C.c_char_p
    L.or_build.restype = P
    L.or_build.argtypes = [C.POINTER(OrParams), C.c_uint64, C.c_double, C.POINTER(C.c_double)]
    L.or_build_explicit.restype = P
    L.or_build_explicit.argtypes = [C.POINTER(OrParams), C.c_uint64, C.POINTER(C.c_int32), C.c_int64,
                                    P, P, P, P]
    L.or_free.argtypes = [P]
    L.or_run.argtypes = [P, C.c_int64]
    L.or_inject.argtypes = [P, P, C.c_int64]
    for name, rt in (("or_num_neurons", C.c_int32), ("or_num_synapses", C.c_int64), ("or_ring_depth", C.c_int32),
                     ("or_step", C.c_int64), ("or_wq_ext", C.c_int32), ("or_num_recorded", C.c_int64),
                     ("or_ring_sum", C.c_double)):
        f = getattr(L, name)
        f.restype, f.argtypes = rt, [P]
    L.or_pop_offsets.argtypes = [P, P]
    L.or_poisson_table.argtypes = [P, C.c_int, P]
    L.or_poisson_count.argtypes = [P, C.c_int64, C.c_int32]
    L.or_constants.argtypes = [P, P]
    L.or_get_csr.argtypes = [P, P, P, P, P, P]
    L.or_get_state.argtypes = [P, P, P, P]
    L.or_set_state.argtypes = [P, P, P, P]
    L.or_get_spikes.argtypes = [P, P, P]
    L.or_clear_spikes.argtypes = [P]
    L.or_get_counters.argtypes = [P, P]
    L.or_philox.argtypes = [P, P, P]
    L.or_round_fp16.restype = C.c_double
    L.or_round_fp16.argtypes = [C.c_double]
    L.or_round_bf16.restype = C.c_double
    L.or_round_bf16.argtypes = [C.c_double]
    L.or_set_threads.argtypes = [C.c_int]
    L.or_max_threads.restype = C.c_int
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr, key):
    """Philox4x64-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def round_fp16(x):
    return lib().or_round_fp16(float(x))


def round_bf16(x):
    return lib().or_round_bf16(float(x))


def set_threads(n):
    lib().or_set_threads(int(n))


def max_threads():
    return lib().or_max_threads()


class OracleNet:
    """One microcircuit instance simulated by the oracle."""

    def __init__(self, handle, params):
        self._h = handle
        self.params = params
        L = lib()
        self.N = L.or_num_neurons(handle)
        self.M = L.or_num_synapses(handle)
        self.R = L.or_ring_depth(handle)
        off = np.zeros(NPOP + 1, dtype=np.int32)
        L.or_pop_offsets(handle, _ptr(off))
        self.pop_offsets = off

    @classmethod
    def build(cls, seed, scale, conn, params=None):
        params = params or default_params()
        conn = np.ascontiguousarray(conn, dtype=np.float64).reshape(64)
        h = lib().or_build(C.byref(params), C.c_uint64(seed), float(scale),
                           conn.ctypes.data_as(C.POINTER(C.c_double)))
        if not h:
            raise RuntimeError("oracle build failed: " + lib().or_last_error().decode())
        return cls(h, params)

    @classmethod
    def build_explicit(cls, pop_sizes, pre, post, w, d, params=None, seed=1):
        params = params or default_params()
        ps = np.ascontiguousarray(pop_sizes, dtype=np.int32)
        pre = np.ascontiguousarray(pre, dtype=np.int32)
        post = np.ascontiguousarray(post, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.int32)
        h = lib().or_build_explicit(C.byref(params), C.c_uint64(seed), ps.ctypes.data_as(C.POINTER(C.c_int32)),
                                    len(pre), _ptr(pre), _ptr(post), _ptr(w), _ptr(d))
        if not h:
            raise RuntimeError("oracle build failed: " + lib().or_last_error().decode())
        return cls(h, params)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_free(self._h)
            self._h = None

    # -- simulation ---------------------------------------------------------
    def run(self, steps):
        if lib().or_run(self._h, int(steps)) != 0:
            raise RuntimeError("oracle run failed: " + lib().or_last_error().decode())

    def inject(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        if lib().or_inject(self._h, _ptr(ids), len(ids)) != 0:
            raise RuntimeError("oracle inject failed: " + lib().or_last_error().decode())

    @property
    def step(self):
        return lib().or_step(self._h)

    # -- inspection ---------------------------------------------------------
    def csr(self):
        L = lib()
        rp = np.zeros(self.N + 1, dtype=np.int64)
        post = np.zeros(self.M, dtype=np.int32)
        wq = np.zeros(self.M, dtype=np.int32)
        d = np.zeros(self.M, dtype=np.uint8)
        w64 = np.zeros(self.M, dtype=np.float64) if self.params.mode == FP64 else None
        L.or_get_csr(self._h, _ptr(rp), _ptr(post), _ptr(wq), _ptr(d), _ptr(w64))
        return dict(row_ptr=rp, post=post, wq=wq, d=d, w64=w64)

    def state(self):
        u = np.zeros(self.N, dtype=np.float64)
        I = np.zeros(self.N, dtype=np.float64)
        r = np.zeros(self.N, dtype=np.int32)
        lib().or_get_state(self._h, _ptr(u), _ptr(I), _ptr(r))
        return u, I, r

    def set_state(self, u=None, I=None, refr=None):
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        I = None if I is None else np.ascontiguousarray(I, dtype=np.float64)
        refr = None if refr is None else np.ascontiguousarray(refr, dtype=np.int32)
        lib().or_set_state(self._h, _ptr(u), _ptr(I), _ptr(refr))

    def spikes(self, clear=False):
        L = lib()
        n = L.or_num_recorded(self._h)
        steps = np.zeros(n, dtype=np.int64)
        ids = np.zeros(n, dtype=np.int32)
        if n:
            L.or_get_spikes(self._h, _ptr(steps), _ptr(ids))
        if clear:
            L.or_clear_spikes(self._h)
        return steps, ids

    def counters(self):
        out = np.zeros(5, dtype=np.int64)
        lib().or_get_counters(self._h, _ptr(out))
        return dict(steps=int(out[0]), spikes=int(out[1]), events=int(out[2]),
                    poisson_events=int(out[3]), max_spikes_per_step=int(out[4]))

    def poisson_table(self, pop):
        out = np.zeros(KMAX, dtype=np.uint64)
        lib().or_poisson_table(self._h, int(pop), _ptr(out))
        return out

    def poisson_count(self, n, i):
        return lib().or_poisson_count(self._h, int(n), int(i))

    def constants(self):
        out = np.zeros(9, dtype=np.float64)
        lib().or_constants(self._h, _ptr(out))
        return dict(P22=out[0], P11=out[1], P21=out[2], P20=out[3],
                    P22f=np.float32(out[4]), P11f=np.float32(out[5]), P21f=np.float32(out[6]),
                    P20f=np.float32(out[7]), theta=out[8])

    def wq_ext(self):
        return lib().or_wq_ext(self._h)

    def ring_sum(self):
        return lib().or_ring_sum(self._h)
