"""Seeded synthetic inputs shared by the simulator tests, the benchmark and the
oracle-side checks.

This module holds none of the simulation's arithmetic: it only generates the
inputs a user would supply -- the 8x8 connection-probability table (a seeded
stand-in for the microcircuit's published table, which is not shipped here),
the scales of an uneven batch, forced spike lists for the delivery
microbenchmark, and stand-in amplitudes for the DC-input workload.
"""
from .conn_table import (FULL_SIZE, K_EXT, POP_NAMES, STANDIN_SEED, standin_conn_table,
                         standin_description)
from .workloads import batch_scales, dc_standin_amplitudes, forced_spike_list, relaxed_start

__all__ = ["FULL_SIZE", "K_EXT", "POP_NAMES", "STANDIN_SEED", "standin_conn_table",
           "standin_description", "batch_scales", "dc_standin_amplitudes", "forced_spike_list", "relaxed_start"]
