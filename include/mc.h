/*
 * mc.h -- C ABI of libmc, a fixed-step simulator of the layered cortical
 * microcircuit (8 populations, 77,169 neurons and ~3e8 synapses at full scale)
 * for AMD Instinct MI355X (gfx950).
 *
 * The model follows Rhodes et al., "Real-Time Cortical Simulation on Neuromorphic
 * Hardware" (arXiv 1909.08665): Sec. 2a and Eq. 1 define the neuron (leaky
 * integrate-and-fire, current-based exponential synapses, reset on threshold
 * crossing), the weight and delay distributions and the Poisson background;
 * Sec. 3a(ii) defines the synaptic matrix (rows indexed by presynaptic neuron,
 * each word = target, weight, delay) and the per-neuron synaptic input buffers
 * (255 slots, the slot for t + delay receives the weight); Sec. 3c defines a
 * synaptic event (one spike reaching one postsynaptic synapse).
 *
 * Each simulation step (dt = 0.1 ms) runs entirely on the GPU:
 *   1. read and clear every neuron's input-buffer slot for this step, add the
 *      step's Poisson background count times the background weight;
 *   2. exact-integration LIF update;
 *   3. threshold test, reset, spike compaction and recording;
 *   4. delivery of each spiking neuron's synaptic row into the targets' delay
 *      ring buffers (int32, 1/256 pA fixed point, integer atomics).
 *
 * Conventions for every call:
 *   - every call returns MC_OK (0) or a negative MC_ERR_* code; on error,
 *     mc_last_error() returns a message (thread-local, valid until the next call
 *     on the same thread); no C++ exception crosses this interface;
 *   - all pointers in the signatures are HOST pointers owned by the caller,
 *     read or written only during the call;
 *   - an mc_net owns all of its device memory and its HIP stream; it is not
 *     thread-safe: one thread at a time per handle;
 *   - neuron ids are instance-local and ordered by population:
 *     L2/3E, L2/3I, L4E, L4I, L5E, L5I, L6E, L6I;
 *   - a spike time is the integer step index n (t = n * dt).
 */
#ifndef MC_H
#define MC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define MC_OK 0
#define MC_ERR_ARG (-1)              /* invalid argument or configuration */
#define MC_ERR_NOMEM (-2)            /* host or device allocation failed */
#define MC_ERR_HIP (-3)              /* a HIP runtime call failed */
#define MC_ERR_OVERFLOW_BOUND (-4)   /* int32 input-buffer bound exceeded at build */
#define MC_ERR_DELAY_RANGE (-5)      /* a delay outside [1, 255] steps */
#define MC_ERR_RECORD_OVERFLOW (-6)  /* device spike recorder overflowed during a run */
#define MC_ERR_BUFFER_TOO_SMALL (-7) /* caller buffer too small; nothing consumed */
#define MC_ERR_IO (-8)               /* checkpoint file could not be read/written */
#define MC_ERR_UNSUPPORTED (-9)      /* requested engine cannot run this network */

/* Synaptic weight store (Sec. 2a weights; reduced-precision forms). */
#define MC_W_FP32 0   /* float weight holding the 1/256 pA fixed-point value */
#define MC_W_FP16 1   /* IEEE binary16, round-to-nearest-even from double */
#define MC_W_BF16 2   /* bfloat16, round-to-nearest-even from double */

/* Step engines.  All give bit-identical results. */
#define MC_ENGINE_AUTO 0    /* TILED when the network fits, else GRAPH */
#define MC_ENGINE_GRAPH 1   /* two kernels per step, K steps captured in a hipGraph */
#define MC_ENGINE_TILED 2   /* persistent kernel, LDS-resident ring per neuron tile */

#define MC_NPOP 8

/*
 * Model and run configuration.  Initialise with mc_config_default(), then set
 * conn_probs (required: the 8x8 table has no default).  Parameter defaults are
 * those of Sec. 2a of the paper with the workload's delay values.
 */
typedef struct mc_config {
    uint32_t struct_size;        /* sizeof(mc_config), set by mc_config_default */
    const double *conn_probs;    /* [64] conn_probs[8*a + b] = probability that a given
                                    (pre in population a, post in population b) pair is
                                    connected; each in [0, 1).  Required. */
    int32_t wfmt;                /* MC_W_FP32 | MC_W_FP16 | MC_W_BF16 */
    int32_t poisson_on;          /* 1: Poisson background drive (default); 0: none */
    int32_t init_mode;           /* 0: u ~ U[0, theta), I = 0 (default); 1: u = I = 0;
                                    2: relaxed start (init_u_*, init_i_* below) */
    int32_t engine;              /* MC_ENGINE_* */
    int64_t record_capacity;     /* device recorder entries; 0 = automatic */
    double full_size[MC_NPOP];   /* full-scale population sizes */
    double k_ext[MC_NPOP];       /* Poisson in-degree per population */
    double i_dc_pa[MC_NPOP];     /* constant input current per population (0) */
    double nu_bg_hz;             /* background rate per source: 8 Hz */
    double dt_ms;                /* 0.1 */
    double tau_m_ms;             /* 10 */
    double c_m_pf;               /* 250 */
    double tau_syn_ms;           /* 0.5 */
    double t_ref_ms;             /* 2 */
    double theta_mv;             /* V_th - E_L = 15 */
    double w_mean_pa;            /* 87.8 */
    double w_sd_pa;              /* 8.78 */
    double g;                    /* inhibitory weight factor: -4 */
    double l4e_l23e_factor;      /* mean factor for L4E -> L2/3E: 2 */
    double w_ext_pa;             /* background weight: 87.8 */
    double d_mean_exc_ms, d_sd_exc_ms;   /* 1.5, 0.75 */
    double d_mean_inh_ms, d_sd_inh_ms;   /* 0.8, 0.4 */
    int32_t device_build;        /* 0: draw and sort the synapses on the host (default);
                                    1: on the GPU -- the same draws and row order, with the
                                    device's log/sqrt/cos/sin (a quantised weight or delay
                                    can differ from the host build's only when its exact
                                    value lies within ~1e-13 of a rounding boundary).
                                    Needs fewer than 2^24 neurons and 2^32 synapses. */
    /* Relaxed start (init_mode 2; Sec. 4a: initial potentials chosen so that the first
       steps already look like the steady state).  Per population: the synaptic current
       I ~ N(init_i_mean_pa, init_i_sd_pa); the potential u from the density of
       N(init_u_mean_mv, init_u_sd_mv) minus its mirror image in the threshold
       (zero at theta, like the steady state's), drawn by rejection from Philox blocks
       (neuron, 1 + attempt, 0, 3).  Needs init_u_sd_mv > 0, init_u_mean_mv < theta. */
    double init_u_mean_mv[MC_NPOP], init_u_sd_mv[MC_NPOP];
    double init_i_mean_pa[MC_NPOP], init_i_sd_pa[MC_NPOP];
} mc_config;

typedef struct mc_counters {
    int64_t steps;               /* steps simulated so far */
    int64_t spikes;              /* spikes emitted (recurrent sources) */
    int64_t events;              /* synaptic events: sum of out-degrees of spiking neurons (Sec. 3c) */
    int64_t poisson_events;      /* background spikes drawn (whole network, all instances) */
    int64_t max_spikes_per_step; /* largest spike count in one step (of `instance`, or of the
                                    whole network for instance = -1) */
    int64_t dropped_events;      /* events not delivered because a step ran past its budget
                                    (mc_set_step_budget); 0 when no budget is set */
} mc_counters;

typedef struct mc_info {
    int32_t n_instances;
    int32_t ring_depth;          /* R: power of two > the largest delay */
    int32_t engine;              /* engine selected for mc_run */
    int32_t wfmt;
    int64_t n_neurons;           /* all instances */
    int64_t n_synapses;          /* all instances */
    int32_t tile_neurons;        /* TILED engine: largest tile, neurons (0 otherwise) */
    int32_t n_tiles;             /* TILED engine: workgroups (tiles never straddle instances) */
    int32_t graph_chunk;         /* GRAPH engine: steps per captured graph */
    int32_t seg;                 /* GRAPH engine: synapses per delivery work item */
    int32_t block;               /* GRAPH engine: threads per block of the neuron kernel */
    int32_t deliver_grid;        /* GRAPH engine: blocks of the delivery kernel */
    int32_t lds_ring;            /* TILED engine: 1 ring in LDS, 0 ring in global memory */
    int32_t syn_bytes;           /* bytes read per delivered synapse by the engine in use:
                                    GRAPH 9 (FP32) / 7 (FP16, BF16) from the CSR arrays;
                                    TILED 8, or 4 for FP16/BF16 tiles of <= 1024 neurons */
    int32_t poll_delay;          /* TILED engine: sleep before a step's first poll of the
                                    other tiles' words, units of 64 clocks */
    int32_t lds_window;          /* TILED engine with the ring in global memory: slots n+1 ..
                                    n+lds_window also kept in LDS (events with delays up to
                                    it are added there); 0 otherwise */
} mc_info;

/* Launch knobs chosen by the autotuner or set by hand (0 = keep current). */
typedef struct mc_launch {
    int32_t engine;
    int32_t tile;                /* TILED engine: at most this many neurons per tile, 16..4096 */
    int32_t ring;                /* TILED engine: 0 auto, 1 ring in LDS, 2 ring in global memory
                                    owned by the tile's workgroup */
    int32_t graph_chunk;         /* 1..1024 */
    int32_t seg;                 /* 64, 128, 256 or 512 */
    int32_t block;               /* 64, 128, 256 or 512 */
    int32_t deliver_grid;        /* >= 1 */
    int32_t poll_delay;          /* TILED engine: sleep before a step's first poll of the other
                                    tiles' words, in units of 64 clocks, 1..255; -1 for none.
                                    Speed only: results do not depend on it. */
    int32_t coop;                /* TILED engine: 1 cooperative launch (the runtime guarantees
                                    that all workgroups are resident at once), 2 ordinary
                                    launch (the default: 15-20 us cheaper per launch) while the
                                    tiles are at most one per compute unit -- with more, the
                                    launch is cooperative either way; relies on no other work
                                    holding the compute units for longer than the wait limit
                                    of mc_set_wait_limit.  Speed only. */
    int32_t lanes;               /* TILED engine: lanes per spike when a step's (or an injection's)
                                    spikes are delivered by a cursor, 1..64 (default: about the
                                    mean sub-row length).  Speed only. */
} mc_launch;

/* Fill *cfg with the defaults of Sec. 2a; conn_probs is left NULL. */
int mc_config_default(mc_config *cfg);

/*
 * Build one microcircuit instance at `scale` (0, 1] from `seed` and upload it.
 * Population sizes are floor(N_full * scale + 0.5) (at least 1).  For each
 * ordered population pair a fixed total of K = log(1-p)/log(1-1/(N_a N_b))
 * synapses (rounded) is drawn with uniform pre and post (multapses allowed),
 * normal weights and delays as in Sec. 2a (delays rounded to steps, clipped to
 * [1, 255], the buffer length of Sec. 3a(ii)); random numbers from
 * Philox4x64-10 keyed (seed, 0).  Untimed set-up.
 * On success *out owns the network; release with mc_free().
 * Errors: MC_ERR_ARG, MC_ERR_NOMEM, MC_ERR_HIP, MC_ERR_OVERFLOW_BOUND.
 */
int mc_build_network(uint64_t seed, double scale, const mc_config *cfg, struct mc_net **out);

/*
 * Build `n` independent instances (seeds[i], scales[i]) as disjoint blocks of one
 * network advanced by the same kernels; instance i behaves exactly as the
 * single network built with (seeds[i], scales[i]).  Errors as mc_build_network.
 */
int mc_build_batch(const uint64_t *seeds, const double *scales, int32_t n,
                   const mc_config *cfg, struct mc_net **out);

/*
 * Advance the network by `steps` steps of dt (Sec. 2a: fixed-step simulation of
 * Eq. 1 at dt = 0.1 ms).  Each step consumes and clears every neuron's input-
 * buffer slot for the step, adds the step's Poisson background (Sec. 3a(ii) and
 * 3a(iii): a count of background spikes per neuron per timer tick), integrates
 * Eq. 1 exactly, records the spikes, and adds every spiking neuron's synaptic row
 * into the targets' slots `delay` steps ahead (Sec. 3a(ii)).
 * Synchronous: returns when the GPU is done.  mc_run(a); mc_run(b) gives
 * bit-identical results to mc_run(a + b).  The step index (steps already run
 * plus `steps`) must stay below 2^31, i.e. about 59.6 h of biological time at
 * dt = 0.1 ms; a longer run is refused with MC_ERR_ARG before anything runs.
 * Errors: MC_ERR_ARG (steps < 0, step limit), MC_ERR_HIP (a HIP call failed, or a
 * workgroup's wait for the other tiles' spikes timed out: the network is then
 * marked failed and every later call on it except mc_load_state, mc_get_info,
 * mc_instance_size, mc_last_error and mc_free returns MC_ERR_HIP until a checkpoint
 * is loaded), MC_ERR_RECORD_OVERFLOW (the spikes that did not fit are lost;
 * counters still count them).
 */
int mc_run(struct mc_net *net, int64_t steps);

/*
 * Copy out and consume the spikes of `instance` recorded since the previous call,
 * sorted by (step, id): the output spike trains from which the paper's results
 * are computed (Sec. 2a: spike trains after the initial transient; Sec. 4b:
 * rates, CV of the inter-spike interval, correlations), a spike at step n meaning
 * V crossed the threshold in that step (Eq. 1).  steps_out/ids_out have room for
 * `cap` entries; *count_out receives the number of spikes.  If cap is too small,
 * returns MC_ERR_BUFFER_TOO_SMALL with *count_out = the number needed and consumes
 * nothing.  Errors: MC_ERR_ARG (NULL pointers, instance out of range).
 */
int mc_get_spikes(struct mc_net *net, int32_t instance, int64_t *steps_out, int32_t *ids_out,
                  int64_t cap, int64_t *count_out);

/*
 * Copy the state of `instance`: the two state variables of Eq. 1 (Sec. 2a) --
 * membrane potential relative to rest, u = V - E_L in mV, and synaptic current
 * I_syn in pA -- and the remaining refractory steps (V held at V_reset for t_ref
 * after a spike).  u_mv, i_pa: float [n]; refr: int32 [n]; host memory owned by
 * the caller; any output pointer may be NULL.  `n` must equal the instance's
 * neuron count.  Errors: MC_ERR_ARG (n or instance wrong), MC_ERR_HIP.
 */
int mc_get_state(struct mc_net *net, int32_t instance, float *u_mv, float *i_pa, int32_t *refr, int64_t n);

/* Overwrite the state of `instance` (same layout as mc_get_state; NULL = keep). */
int mc_set_state(struct mc_net *net, int32_t instance, const float *u_mv, const float *i_pa,
                 const int32_t *refr, int64_t n);

/*
 * Counters of `instance` over the spikes recorded so far: steps, spikes,
 * synaptic events -- one spike reaching one postsynaptic synapse (Sec. 3c),
 * i.e. the sum of the out-degrees of the spiking neurons, recurrent only --,
 * background (Poisson) spikes drawn (Sec. 3a(iii)) and the largest spike count
 * of one step.  instance = -1 gives the whole network; poisson_events is always
 * the whole-network value.  *out is caller-owned host memory.
 * Errors: MC_ERR_ARG (NULL pointer, instance out of range), MC_ERR_HIP.
 */
int mc_get_counters(struct mc_net *net, int32_t instance, mc_counters *out);

/* Sizes and the launch configuration in use. */
int mc_get_info(struct mc_net *net, mc_info *out);

/*
 * Copy the synapse store of `instance` back from the GPU, with instance-local
 * target ids: row_ptr [N+1] (int64), post [M], wq [M] (weight in 1/256 pA as
 * int32), d [M] (delay in steps).  Rows are ordered by presynaptic neuron.
 * Any output may be NULL.  `n_synapses` must equal the instance's synapse count.
 */
int mc_get_csr(struct mc_net *net, int32_t instance, int64_t *row_ptr, int32_t *post, int32_t *wq,
               uint8_t *d, int64_t n_synapses);

/* Number of neurons and synapses of `instance`. */
int mc_instance_size(struct mc_net *net, int32_t instance, int64_t *n_neurons, int64_t *n_synapses);

/*
 * External stimulation: deliver the synaptic rows of the `count` neurons `ids`
 * (instance-local) of `instance` as if they had spiked in the last completed
 * step -- each synapse adds its weight into its target's input-buffer slot
 * `delay` steps later (Sec. 3a(ii)), so the next mc_run sees them.  The
 * injected spikes are not recorded and not counted.  *events_out (may be NULL)
 * receives the number of synapses delivered.  Errors: MC_ERR_ARG (bad id).
 */
int mc_inject_spikes(struct mc_net *net, int32_t instance, const int32_t *ids, int64_t count, int64_t *events_out);

/*
 * mc_inject_spikes for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same delivery, with the ids staged in a fixed device array of
 * 1,048,576 entries that the library holds per GPU from the first network
 * built on it until the process ends (resolved at that build), instead of a
 * buffer allocated on first use.  Allocates nothing; synchronous like
 * mc_inject_spikes.  Every call on one GPU shares that array, so calls that
 * overlap on one GPU (from several threads or processes' networks on it) race.
 * Errors: as mc_inject_spikes, and MC_ERR_ARG when count exceeds 1,048,576.
 */
int mc_inject_spikes_noalloc(struct mc_net *net, int32_t instance, const int32_t *ids, int64_t count,
                             int64_t *events_out);

/* Select launch knobs (engine, tile size, graph chunk, work-item size, block, grid).
   MC_ERR_UNSUPPORTED if the TILED engine cannot hold the network (LDS, co-residency). */
int mc_set_launch(struct mc_net *net, const mc_launch *l);

/*
 * Autotuner: time each candidate launch configuration (the one in use first)
 * twice for `trial_steps` steps on a saved copy of the state, restore the state,
 * and keep the fastest; another configuration replaces the one in use only when
 * at least 3 % faster.  Results of later runs do not depend on the choice.
 * Errors: MC_ERR_ARG (trial_steps outside [1, 100000]), MC_ERR_HIP (a trial
 * failed: the configuration and state from before the call are restored).
 */
int mc_tune(struct mc_net *net, int64_t trial_steps);

/* Use the caller's HIP stream (hipStream_t passed as void*); NULL = own stream. */
/*
 * Lossy real-time mode (Sec. 3a(iii) and 4a: a core that has not finished a
 * step's synaptic processing when the next timer tick comes drops what is left
 * and counts it).  With budget_us > 0 every tile of the TILED engine stops
 * delivering a step's spikes once budget_us has passed since it started that
 * step; the events it did not deliver are dropped and counted in
 * mc_counters.dropped_events.  Results then depend on timing and no longer
 * match a run without a budget.  budget_us = 0 (the default) turns it off.
 * Errors: MC_ERR_ARG (negative or above 20,000,000 us); mc_run returns
 * MC_ERR_UNSUPPORTED on the GRAPH engine while a budget is set.
 */
int mc_set_step_budget(struct mc_net *net, double budget_us);

int mc_set_stream(struct mc_net *net, void *hip_stream);

/*
 * Kernel timing with HIP events on the network's stream: enable (1) or disable (0)
 * timing of the dominant kernel; mc_get_timing returns the summed duration in ms
 * and the number of launches timed since it was enabled.  Enabling records and
 * queries each of the library's event pairs once (waiting for the network's
 * stream), so that their first-use cost falls outside the runs it times.
 */
int mc_set_timing(struct mc_net *net, int32_t on);
int mc_get_timing(struct mc_net *net, double *kernel_ms, int64_t *launches);

/*
 * Per-step latency record of the TILED engine (the paper's true-real-time
 * criterion, Sec. 2c and 3a(iii): every step must finish within its period).
 * mc_set_trace(net, k) records, for the first k steps of the next mc_run, eight
 * words per (step, tile) from the GPU's constant 100 MHz clock: step start,
 * spikes published, barrier arrival, next Poisson draw done, barrier passed,
 * spike counts gathered, delivery done, and the step's spike count; then one
 * more row per tile with the launch's own timestamps: kernel entry, start of
 * the first step (after the ring and state are loaded), end of the last step,
 * end of the write-back, then within the write-back: state stored, ring
 * stored, counters added.  k = 0 disables it.  mc_get_trace copies
 * [k + 1][n_tiles][8] words into `out` (cap entries) and sets *count;
 * MC_ERR_BUFFER_TOO_SMALL if cap is too small.
 */
int mc_set_trace(struct mc_net *net, int32_t steps);
int mc_get_trace(struct mc_net *net, uint64_t *out, int64_t cap, int64_t *count);

/*
 * Checkpoint: write / read the full dynamic state (step counter, neuron state,
 * input buffers, counters and unread spikes) to / from `path`.  The random
 * streams are counter-based, so a restored run continues bit-identically.
 * mc_load_state requires a network built with the same arguments.
 */
int mc_save_state(struct mc_net *net, const char *path);
int mc_load_state(struct mc_net *net, const char *path);

/*
 * Delivery-path counters of the TILED engine (which code path delivered each
 * step's spikes), summed over tiles and steps since the network was built:
 * counts[k] for k < n (entries beyond the ones defined are 0):
 *   0 steps without spikes;  1 ids from the tile words, fixed lane groups per
 *   spike;  2 ids from the tile words, events spread by a length scan;  3 one
 *   spike per thread, ids looked up;  4 more spikes than threads;  5 spike
 *   batches after the first (steps of more than 2048 spikes);  6 looked-up ids
 *   placed by the per-tile map;  7 placed by a binary search;  8 some tile sent
 *   more spikes than its exchange word carries (ids read from entry words).
 * Counts are per tile and step (and batch).  For coverage checks; results do
 * not depend on the path.  Errors: MC_ERR_ARG, MC_ERR_HIP.
 */
int mc_get_paths(struct mc_net *net, int64_t *counts, int32_t n);

/*
 * Bound on a cross-tile wait of the TILED engine: a workgroup that has polled
 * another tile's spike word `polls` times (checked every 1024 polls) without
 * seeing it gives up, and so does every other workgroup of the launch; mc_run
 * then returns MC_ERR_HIP and the network is marked failed (see mc_run).
 * Default 2^24 polls (seconds of waiting: a wait that long means the launch
 * cannot complete).  polls = 0 makes every wait give up at once -- for testing
 * the failure path without a real fault.  Errors: MC_ERR_ARG (polls outside
 * [0, 2^32 - 1]).
 */
int mc_set_wait_limit(struct mc_net *net, int64_t polls);

/*
 * Ceilings of the memory system the step kernels run against, measured on the
 * current device (no network needed).  The delivery of Sec. 3a(ii) adds each
 * event's weight into a ring slot with an integer atomic and streams the
 * synaptic rows from HBM, so these bound it:
 *   MC_PROBE_HBM_COPY       streaming copy of `bytes` (half read, half written):
 *                           *rate in GB/s;
 *   MC_PROBE_LDS_ATOMICS    int32 atomic adds at random LDS words in every
 *                           compute unit (the tiled engine's ring): atomics/s;
 *                           `bytes` ignored;
 *   MC_PROBE_DEVICE_ATOMICS device-scope int32 atomic adds at random words of a
 *                           `bytes` buffer (L2-, Infinity-Cache- or HBM-resident
 *                           by size; the global-ring and graph forms): atomics/s;
 *   MC_PROBE_HBM_GATHER     reads of whole 128-byte cache lines at random
 *                           places of a `bytes` buffer, by groups of 16 lanes
 *                           (the unit in which sub-row reads at random places
 *                           reach HBM): GB/s.
 * *kernel_ms (may be NULL) receives the timed launch's duration.  Allocates and
 * frees its own device buffers.  Errors: MC_ERR_ARG (unknown kind, bytes outside
 * [8 KiB, 64 GiB]), MC_ERR_NOMEM, MC_ERR_HIP.
 */
#define MC_PROBE_HBM_COPY 0
#define MC_PROBE_LDS_ATOMICS 1
#define MC_PROBE_DEVICE_ATOMICS 2
#define MC_PROBE_HBM_GATHER 3
int mc_probe(int32_t kind, int64_t bytes, double *rate, double *kernel_ms);

/* Release the network and all of its device memory.  NULL is allowed. */
void mc_free(struct mc_net *net);

/* Message of the last error on this thread ("" if none). */
const char *mc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MC_H */
