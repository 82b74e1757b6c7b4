// kernels.hpp -- device-side view of a network and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mc {

constexpr int kPoisMaxDev = 24;
constexpr uint64_t kMask40 = (uint64_t{1} << 40) - 1;
constexpr uint32_t kFlagRecordOverflow = 1u;

// Control words of the step loop, in device memory.
struct StepCtl {
    int64_t nbase;                    // step index at the start of the current launch chunk
    int64_t rec_total;                // spikes recorded since the last drain
    unsigned long long cnt[3];        // per step (n % 3): spikes << 40 | delivery work items
    unsigned long long events;        // recurrent synaptic events
    int32_t max_s;                    // largest spike count of one step
    uint32_t flags;
};

// Everything a kernel needs, passed by value.
struct DevNet {
    int32_t n;                        // neurons (all instances)
    int32_t ring_mask;                // R - 1, R a power of two
    int32_t ref_steps;
    int32_t wq_ext;
    float p22, p11, p21, theta;
    int32_t poisson_on;
    int32_t seg;                      // synapses per delivery work item
    int32_t wfmt;
    int32_t pad0;
    // neuron state and description
    float *u;
    float *cur;                       // synaptic current I
    uint8_t *refr;
    const uint32_t *meta;             // (instance << 3) | population
    const int32_t *inst_off;          // [instances + 1]
    const uint64_t *seeds;            // [instances]
    const float *cdc;                 // [8] P20 * I_dc
    const uint64_t *pois_thr;         // [8 * 24]
    int32_t *ring;                    // [R][n]
    // synapse store, CSR by presynaptic neuron
    const uint64_t *row_ptr;          // [n + 1]
    const int32_t *tgt;               // [m] global target id
    const void *w;                    // [m] float, or 16-bit FP16/BF16 bits
    const uint8_t *dly;               // [m] delay in steps
    // step loop
    StepCtl *ctl;
    uint64_t *work;                   // delivery work items: pre << 32 | chunk
    unsigned long long *pois_acc;     // per-block Poisson event sums
    uint64_t *rec;                    // spike recorder: step << 32 | neuron id
    int64_t rec_cap;
};

// Spike record entry: step index (< 2^31) in the high word, global neuron id in the low.
__host__ __device__ inline uint64_t rec_entry(int64_t step, int32_t id)
{
    return (static_cast<uint64_t>(static_cast<uint32_t>(step)) << 32) | static_cast<uint32_t>(id);
}

// Head of a spike-recorder buffer (the entries follow it): the counters of the
// tiled launch that records into it.  Launches alternate between two buffers
// and each launch zeroes the other buffer's head, so the host clears nothing
// between launches and copies one head plus entries per launch.
struct RecHead {
    unsigned long long rec_total;     // spikes recorded by the launch
    uint32_t flags;                   // kFlag* of the launch
    uint32_t pad[13];                 // 64 bytes
};

// Tiled persistent engine.  Tiles are ranges of consecutive neurons that never
// straddle two instances; a tile's workgroup exchanges spikes only with the
// tiles of its own instance.
struct TileDesc {
    int32_t t0;                       // first neuron (global id)
    int32_t len;                      // neurons in the tile
    int32_t itile0;                   // first tile of this tile's instance
    int32_t intiles;                  // number of tiles of the instance
    int32_t inst_n0;                  // first neuron of the instance
    int32_t stride;                   // nominal tile length of the instance: tile k starts at inst_n0 + k * stride
    int64_t sub_base;                 // `subrow` entry of (presynaptic p, this tile) is sub_base + p * intiles
};

// Packed synapse records of the tiled engine, in CSR order (so a sub-row is a
// contiguous index range): tile-local target, delay, weight.
//   0: 8 B {u16 target | u8 delay | u8 0, f32 weight}
//   1: 8 B {same, FP16 weight bits}          2: 8 B {same, BF16 weight bits}
//   3: 4 B {10-bit target | 6-bit delay | FP16 weight}   (tile <= 1024, R <= 64)
//   4: 4 B {10-bit target | 6-bit delay | BF16 weight}
enum SynFmt : int32_t { kSyn8F32 = 0, kSyn8F16 = 1, kSyn8BF16 = 2, kSyn4F16 = 3, kSyn4BF16 = 4 };

struct TiledNet {
    DevNet base;
    int32_t n_tiles;
    int32_t tile_max;                 // largest tile (LDS / entry stride)
    int32_t max_intiles;              // most tiles of one instance
    int32_t tile_offset;              // injection: first tile of the launch
    const TileDesc *tiles;            // [n_tiles]
    const uint2 *subrow;              // per instance: [its neurons][its tiles] (first synapse, count) of the
                                      // sub-row of that presynaptic neuron that targets the tile
    const void *syn;                  // packed synapse records (SynFmt), CSR order
    int32_t syn_fmt;
    int32_t poll_delay;               // sleep before the first poll of a step, in units of 64 clocks
    uint64_t *xchg;                   // [2][n_tiles] per-step tile words (tag | count | first three offsets)
    uint64_t *xent;                   // [2][n_tiles][tile_max] further spike ids (tag32 | id)
    RecHead *head;                    // this launch's recorder head (entries: base.rec)
    RecHead *head_other;              // the other buffer's head, zeroed for the next launch
    uint32_t *abort_word;             // epoch of a launch in which a wait gave up
    uint32_t epoch;                   // launch number (never 0): the abort word names the launch
    uint32_t spin_limit;              // polls before a wait gives up (0: at once)
    uint64_t *trace;                  // optional [trace_steps][n_tiles][8] phase timestamps
    int32_t trace_steps;
    int32_t gstride;                  // global-ring variant: ints per slot row (multiple of 32)
    unsigned long long *dropped;      // [n_tiles] events dropped by the step budget in this launch
    unsigned long long *paths;        // [kPaths] tile-steps per delivery path, summed over launches
    uint32_t budget_ticks;            // step budget in 100 MHz clock ticks; 0: none
    int32_t win;                      // global-ring variant: LDS window of the nearest `win` slots (< R)
    int32_t lanes;                    // lanes per spike when a step's spikes are delivered with a cursor
                                      // (about the mean sub-row length)
    int32_t *gring;                   // global-ring variant: [n_tiles][R][gstride], one slice per workgroup
};

constexpr int kTraceSlots = 8;             // timestamps per (step, tile)

// Delivery paths of the tiled step kernel, counted per tile and step (a step
// with several spike batches counts each batch).
enum DeliveryPath : int {
    kPathNoSpikes = 0,      // no spike in the instance this step
    kPathGrouped = 1,       // ids from the tile words, fixed lane groups per spike
    kPathFast = 2,          // ids from the tile words, events spread by a length scan
    kPathPerThread = 3,     // one spike per thread: ids looked up, sub-row read here
    kPathBatched = 4,       // more spikes than threads: looked up in a strided loop
    kPathExtraBatch = 5,    // a spike batch after the first (more than 2048 spikes)
    kPathDirectMap = 6,     // looked-up ids placed by the per-tile map
    kPathSearch = 7,        // looked-up ids placed by a binary search over the tile offsets
    kPathEntryWords = 8,    // some tile sent more spikes than its word carries
    kPaths = 9
};

constexpr uint32_t kFlagTimeout = 2u;      // a cross-tile wait gave up
constexpr uint32_t kSpinLimitDefault = 1u << 24;   // polls before a cross-tile wait gives up

hipError_t launch_neuron(const DevNet &d, int block, int s_off, hipStream_t st);
hipError_t launch_deliver(const DevNet &d, int grid, int s_off, hipStream_t st);
hipError_t launch_advance(const DevNet &d, int steps, hipStream_t st);
hipError_t launch_clear_i32(int32_t *p, int64_t n, hipStream_t st);

// Tiled engine: one cooperative launch advances `steps` steps.  `lds_ring`
// selects the ring in LDS (true) or in global memory owned by the tile's
// workgroup; `npt` neurons per thread (1, 2 or 4).
struct TiledShape {
    bool lds_ring;
    int npt;
    int threads;
    int win;                          // global-ring variant: LDS window rows
    size_t lds;                       // dynamic LDS bytes
};
TiledShape tiled_shape(int tile_max, int max_intiles, int ring, bool lds_ring, int win = 0);
// coop: a cooperative launch (the runtime guarantees that every workgroup is
// resident); otherwise an ordinary launch, which relies on the occupancy check
// done at set-up and on nothing else occupying the device's compute units
// indefinitely (the waits are bounded either way).
hipError_t launch_tiled(const TiledNet &t, const TiledShape &sh, int64_t steps, bool coop, hipStream_t st);
hipError_t tiled_max_coresident(int wfmt, const TiledShape &sh, int *blocks_per_cu);
// Spike injection (external stimulation): deliver the rows of `ids` as if they
// spiked in step n-1.  Tiled form needs the tile ring to fit in LDS; it
// takes the spikes in batches of inject_batch() (as many as fit in LDS beside
// the staged ring, a multiple of 256; 0: the ring leaves no room for 256).
int inject_batch(int tile_max, int ring);
size_t inject_lds_bytes(int tile_max, int ring);
// ids: device array of instance-local ids; id_offset: the instance's first global id.
hipError_t launch_inject_tiled(const TiledNet &tn, int first_tile, int ntiles, int threads, const int32_t *ids,
                               int32_t count, int32_t id_offset, int64_t n, hipStream_t st);
hipError_t launch_inject_global(const DevNet &d, const int32_t *ids, int32_t count, int32_t id_offset, int64_t n,
                                hipStream_t st);
// Device-side construction of the tiled engine's sub-row table and packed
// synapse store (rows sorted by target; tile_of: tile index of every neuron).
// Copy a recorder's head and first min(rec_total, n) entries into pinned host
// memory (h_head, h_rec: device addresses of the pinned buffer).
hipError_t launch_copy_out(const RecHead *head, const uint64_t *rec, int64_t n, RecHead *h_head, uint64_t *h_rec,
                           hipStream_t st);
hipError_t launch_subrows(const DevNet &d, const TileDesc *tiles_dev, int n_tiles, int64_t n_neurons, uint2 *subrow,
                          hipStream_t st);
hipError_t launch_pack_synapses(const DevNet &d, const TileDesc *tiles_dev, const int32_t *tile_of, int64_t m,
                                int syn_fmt, void *syn, hipStream_t st);

// Ceilings of the memory system (probe.hip): kind kProbeHbmCopy streams a copy
// of `bytes` (rate in GB/s of bytes read + written), kProbeLdsAtomics does LDS
// int32 atomic adds at random addresses in every compute unit, and
// kProbeDeviceAtomics does device-scope int32 atomic adds at random words of a
// `bytes` buffer (rates in operations per second), and kProbeHbmGather reads
// whole 128-byte lines at random places of a `bytes` buffer (GB/s).  Each times its
// second launch with HIP events.
enum ProbeKind : int { kProbeHbmCopy = 0, kProbeLdsAtomics = 1, kProbeDeviceAtomics = 2, kProbeHbmGather = 3 };
hipError_t run_probe(int kind, int64_t bytes, double *rate, double *kernel_ms);

}  // namespace mc
