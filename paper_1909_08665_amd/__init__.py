"""MI355X-native simulator of the layered cortical microcircuit (fixed 0.1 ms
step: Poisson background, exact-integration LIF, spike compaction, delayed
synaptic delivery into int32 ring buffers), after Rhodes et al.,
"Real-Time Cortical Simulation on Neuromorphic Hardware" (arXiv 1909.08665).

The compute path is libmc.so (hand-written HIP kernels for gfx950 behind the
C ABI in include/mc.h); this package is its Python binding.
"""
from ._binding import (ENGINE_AUTO, ENGINE_GRAPH, ENGINE_TILED, EXPORTS, LIB_PATH, PROBE_DEVICE_ATOMICS,
                       PROBE_HBM_COPY, PROBE_HBM_GATHER, PROBE_LDS_ATOMICS, MCError, Network, W_BF16, W_FP16, W_FP32, lib,
                       make_config, probe)

__all__ = ["Network", "MCError", "lib", "make_config", "LIB_PATH", "EXPORTS",
           "W_FP32", "W_FP16", "W_BF16", "ENGINE_AUTO", "ENGINE_GRAPH", "ENGINE_TILED", "probe",
           "PROBE_HBM_COPY", "PROBE_HBM_GATHER", "PROBE_LDS_ATOMICS", "PROBE_DEVICE_ATOMICS"]
