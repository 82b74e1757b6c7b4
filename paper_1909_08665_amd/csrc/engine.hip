// engine.hip -- device store, step engines and the C ABI of libmc.
//
// The GRAPH engine captures K steps (neuron kernel + delivery kernel per step,
// then a one-thread counter advance) in a hipGraph and replays it; the step
// index lives in device memory, so the spike count never returns to the host
// inside a run.  The TILED engine advances a whole segment of steps in one
// cooperative persistent launch.  Both keep the dynamic state (u, I, refractory
// counts, the [R][N] ring, step index) in the same global arrays between
// launches, so engines can be switched between runs.  The host drains the spike
// recorder between segments, sized so the recorder stays at most a quarter full.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/mc.h"
#include "devbuild.hpp"
#include "kernels.hpp"
#include "model.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define LIVE_OR_FAIL(net)                                                                      \
    do {                                                                                       \
        if ((net)->failed)                                                                     \
            return fail(MC_ERR_HIP, "the network failed in an earlier run (" + (net)->fail_msg +   \
                                        "); load a checkpoint to continue");                   \
    } while (0)

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(MC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

constexpr int64_t kSegMin = 100, kSegMax = 10000;   // steps between recorder drains
constexpr int64_t kAbsorbSerial = 4096;             // records folded in on the calling thread alone
constexpr size_t kUnreadPrefault = 16384;           // spike-list entries per network allocated and touched at build
constexpr double kTuneMargin = 0.03;                // the autotuner switches only for a gain this large
// Tile words carry (n mod 32767) + 1: words left by earlier launches can be
// taken for a new launch's only if the step index jumped ahead by about 2^15.
constexpr int64_t kTagSafe = 32767 - kSegMax - 8;
// Tiled engine: sleep before a step's first poll, in units of 64 clocks, when
// the instances have at least kPollDelayTiles tiles (T tiles each polling T
// words congest the lines the last stores go to); none for fewer tiles.
constexpr int kPollDelayDefault = 32, kPollDelayTiles = 64;

// Staging of the ids of mc_inject_spikes_noalloc, for callers that cannot
// allocate: a file-scope device array (each GPU holds its own copy until the
// process ends), shared by every such call on that GPU, so calls that overlap
// on one GPU race.  Host code uses its device address, resolved once per
// device (device_staging), never the array's name.
constexpr int64_t kNoAllocIds = int64_t{1} << 20;
__device__ __align__(256) int32_t scratch[kNoAllocIds];
constexpr int kMaxDevices = 64;

// Device address of `scratch` on `device`, resolved with that device current
// on the first call for it.
int device_staging(int device, int32_t **out)
{
    static std::mutex mu;
    static int32_t *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return fail(MC_ERR_UNSUPPORTED, "device index beyond the staging table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) hipSetDevice(cur);
        if (e != hipSuccess) return fail(MC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[device] = static_cast<int32_t *>(p);
    }
    *out = addr[device];
    return MC_OK;
}

}  // namespace

struct mc_net {
    mc::ModelParams params{};
    mc::StepConstants sc{};
    mc::HostNet host;                  // host copy: sizes, offsets, row pointers

    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;

    // device buffers
    float *u = nullptr, *cur = nullptr;
    uint8_t *refr = nullptr;
    uint32_t *meta = nullptr;
    int32_t *inst_off = nullptr;
    uint64_t *seeds = nullptr;
    float *cdc = nullptr;
    uint64_t *pois_thr = nullptr;
    int32_t *ring = nullptr;
    uint64_t *row_ptr = nullptr;
    int32_t *tgt = nullptr;
    void *w = nullptr;
    uint8_t *dly = nullptr;
    mc::StepCtl *ctl = nullptr;
    uint64_t *work = nullptr;
    unsigned long long *pois_acc = nullptr;
    int64_t pois_slots = 0;
    // Two spike recorders and their pinned host copies, each a 64-byte head
    // (mc::RecHead: the counters of the tiled launch that used it) followed by
    // the entries (step << 32 | id): the tiled engine alternates them between
    // segments and drains one while the next segment runs, with one copy of the
    // head and entries per launch; the graph engine uses the first's entries.
    void *rblk[2] = {};
    void *h_rblk[2] = {};
    uint64_t *rec[2] = {};            // entries of rblk[b]
    uint64_t *h_rec[2] = {};          // entries of h_rblk[b]
    void *hd_rblk[2] = {};            // device addresses of h_rblk[b]
    int64_t rec_cap = 0;
    mc::StepCtl *h_ctl = nullptr;
    hipStream_t copy_stream = nullptr;
    hipEvent_t seg_ev0[2] = {}, seg_ev1[2] = {}, snap_ev[2] = {};

    // tiled engine
    int tile = 0, n_tiles = 0, tile_max = 0, max_intiles = 0;
    mc::TiledShape tiled_shape{};
    mc::TileDesc *tiles_dev = nullptr;
    int32_t *gring = nullptr;          // private tile rings of the global-ring variant
    int32_t gstride = 0;
    std::vector<mc::TileDesc> tiles_host;
    int32_t *inject_buf = nullptr;     // device copy of injected spike ids
    int32_t *noalloc_ids = nullptr;    // this device's staging array for mc_inject_spikes_noalloc
    int64_t inject_cap = 0;
    uint2 *subrow = nullptr;           // tiled engine: per-tile (first synapse, count) of each sub-row
    void *syn = nullptr;               // tiled engine: packed synapse records
    int32_t syn_fmt = 0;
    uint64_t *xchg = nullptr;
    uint64_t *xent = nullptr;
    unsigned long long *dropped = nullptr;       // [2][n_tiles] events dropped by the step budget, per buffer
    unsigned long long *h_dropped = nullptr;     // pinned copy (copied only while a budget is set)
    uint32_t *abort_word = nullptr;              // epoch of a launch in which a wait gave up
    unsigned long long *paths = nullptr;         // [kPaths] tile-steps per delivery path
    uint32_t budget_ticks = 0;                   // step budget, 100 MHz ticks; 0: none
    int64_t xent_high = 0;            // entry words may carry tags of steps below this
    int64_t xchg_high = 0;            // tile words carry tags of steps below this
    bool exch_dirty = true;           // tile words and counters must be cleared before the next launch
    int next_buf = 0;                 // recorder buffer of the next launch
    uint32_t epoch = 0;               // launches so far (the abort word names a launch)
    uint32_t spin_limit = mc::kSpinLimitDefault;
    double rec_rate = 64.0;           // spikes per step of the last segment (recorder copy size)
    uint64_t *trace = nullptr;
    int32_t trace_steps = 0;
    int32_t trace_tiles = 0;
    int n_cu = 0;
    size_t lds_limit = 0;

    // launch configuration
    int64_t seg_steps = 1000;
    int engine = MC_ENGINE_GRAPH;
    int graph_chunk = 50;
    int seg = 256;
    int block = 256;
    int deliver_grid = 1024;
    int poll_delay = 0;
    bool poll_delay_set = false;      // chosen by mc_set_launch or the tuner; otherwise by tile count
    bool coop = false;                // tiled engine: cooperative launch (else ordinary)
    int lanes = 16;                   // tiled engine: lanes per spike for cursor delivery
    bool lanes_set = false;           // chosen by mc_set_launch; otherwise from the mean sub-row length
    hipGraphExec_t graph_exec = nullptr;
    int graph_k = 0;

    // host-side run state
    int64_t step = 0;
    std::vector<std::vector<std::pair<int64_t, int32_t>>> unread;   // per instance
    // unread[j][0 .. counted[j]) have their out-degrees in inst_events[j]; the
    // rest are counted when the counters, the spikes or a snapshot are read
    std::vector<size_t> counted;
    std::vector<int64_t> inst_spikes, inst_events, inst_max_step;
    std::vector<int32_t> absorb_scratch;            // per-step spike counts of a short record
    std::vector<int64_t> inst_dropped;  // events dropped by the step budget, per instance
    int64_t max_step_spikes = 0;
    int64_t steps_in_flight = 0;      // steps of the segment being drained
    bool overflow = false;
    // Set when a run failed part-way (a HIP error or an abandoned cross-tile
    // wait): the state is then inconsistent, and calls that read or advance it
    // are refused until a checkpoint is loaded.
    bool failed = false;
    std::string fail_msg;

    // kernel timing
    bool timing = false;
    double kernel_ms = 0.0;
    int64_t launches = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

template <class T>
int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) return fail(MC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    return MC_OK;
}

mc::DevNet dev_view(const mc_net *nt)
{
    mc::DevNet d{};
    d.n = static_cast<int32_t>(nt->host.n);
    d.ring_mask = nt->host.ring - 1;
    d.ref_steps = nt->sc.ref_steps;
    d.wq_ext = nt->sc.wq_ext;
    d.p22 = nt->sc.p22;
    d.p11 = nt->sc.p11;
    d.p21 = nt->sc.p21;
    d.theta = nt->sc.theta;
    d.poisson_on = nt->params.poisson_on;
    d.seg = nt->seg;
    d.wfmt = nt->params.wfmt;
    d.u = nt->u;
    d.cur = nt->cur;
    d.refr = nt->refr;
    d.meta = nt->meta;
    d.inst_off = nt->inst_off;
    d.seeds = nt->seeds;
    d.cdc = nt->cdc;
    d.pois_thr = nt->pois_thr;
    d.ring = nt->ring;
    d.row_ptr = nt->row_ptr;
    d.tgt = nt->tgt;
    d.w = nt->w;
    d.dly = nt->dly;
    d.ctl = nt->ctl;
    d.work = nt->work;
    d.pois_acc = nt->pois_acc;
    d.rec = nt->rec[0];
    d.rec_cap = nt->rec_cap;
    return d;
}

void release(mc_net *nt)
{
    if (!nt) return;
    if (nt->graph_exec) hipGraphExecDestroy(nt->graph_exec);
    // Nothing may still run on the streams when their buffers go.
    if (nt->stream) hipStreamSynchronize(nt->stream);
    if (nt->copy_stream) hipStreamSynchronize(nt->copy_stream);
    void *bufs[] = {nt->u, nt->cur, nt->refr, nt->meta, nt->inst_off, nt->seeds, nt->cdc, nt->pois_thr,
                    nt->ring, nt->row_ptr, nt->tgt, nt->w, nt->dly, nt->ctl, nt->work, nt->pois_acc,
                    nt->rblk[0], nt->rblk[1], nt->subrow, nt->syn, nt->xchg, nt->xent, nt->dropped, nt->abort_word,
                    nt->trace, nt->paths, nt->tiles_dev, nt->gring, nt->inject_buf};
    for (void *b : bufs)
        if (b) hipFree(b);
    for (void *b : {nt->h_rblk[0], nt->h_rblk[1], static_cast<void *>(nt->h_ctl), static_cast<void *>(nt->h_dropped)})
        if (b) hipHostFree(b);
    if (nt->ev0) hipEventDestroy(nt->ev0);
    if (nt->ev1) hipEventDestroy(nt->ev1);
    for (int b = 0; b < 2; ++b)
        for (hipEvent_t e : {nt->seg_ev0[b], nt->seg_ev1[b], nt->snap_ev[b]})
            if (e) hipEventDestroy(e);
    if (nt->copy_stream) hipStreamDestroy(nt->copy_stream);
    if (nt->stream && nt->own_stream) hipStreamDestroy(nt->stream);
    delete nt;
}

int params_from_config(const mc_config *cfg, mc::ModelParams &p)
{
    if (!cfg) return fail(MC_ERR_ARG, "cfg must not be NULL (the connection table has no default)");
    if (cfg->struct_size != sizeof(mc_config)) return fail(MC_ERR_ARG, "cfg->struct_size mismatch (use mc_config_default)");
    if (cfg->device_build != 0 && cfg->device_build != 1) return fail(MC_ERR_ARG, "device_build must be 0 or 1");
    if (!cfg->conn_probs) return fail(MC_ERR_ARG, "cfg->conn_probs is required");
    if (cfg->wfmt < MC_W_FP32 || cfg->wfmt > MC_W_BF16) return fail(MC_ERR_ARG, "unknown weight format");
    if (cfg->engine < MC_ENGINE_AUTO || cfg->engine > MC_ENGINE_TILED) return fail(MC_ERR_ARG, "unknown engine");
    if (!(cfg->dt_ms > 0) || !(cfg->tau_m_ms > 0) || !(cfg->tau_syn_ms > 0) || !(cfg->c_m_pf > 0))
        return fail(MC_ERR_ARG, "time constants, capacitance and dt must be positive");
    if (cfg->tau_m_ms == cfg->tau_syn_ms) return fail(MC_ERR_ARG, "tau_m must differ from tau_syn");
    std::memcpy(p.conn, cfg->conn_probs, sizeof(p.conn));
    std::memcpy(p.full_size, cfg->full_size, sizeof(p.full_size));
    std::memcpy(p.k_ext, cfg->k_ext, sizeof(p.k_ext));
    std::memcpy(p.i_dc, cfg->i_dc_pa, sizeof(p.i_dc));
    p.nu_bg_hz = cfg->nu_bg_hz;
    p.dt_ms = cfg->dt_ms;
    p.tau_m_ms = cfg->tau_m_ms;
    p.c_m_pf = cfg->c_m_pf;
    p.tau_syn_ms = cfg->tau_syn_ms;
    p.t_ref_ms = cfg->t_ref_ms;
    p.theta_mv = cfg->theta_mv;
    p.w_mean_pa = cfg->w_mean_pa;
    p.w_sd_pa = cfg->w_sd_pa;
    p.g = cfg->g;
    p.l4e_l23e_factor = cfg->l4e_l23e_factor;
    p.w_ext_pa = cfg->w_ext_pa;
    p.d_mean_exc_ms = cfg->d_mean_exc_ms;
    p.d_sd_exc_ms = cfg->d_sd_exc_ms;
    p.d_mean_inh_ms = cfg->d_mean_inh_ms;
    p.d_sd_inh_ms = cfg->d_sd_inh_ms;
    p.wfmt = cfg->wfmt;
    p.poisson_on = cfg->poisson_on ? 1 : 0;
    p.init_mode = cfg->init_mode;
    if (p.init_mode < 0 || p.init_mode > 2) return fail(MC_ERR_ARG, "init_mode must be 0, 1 or 2");
    std::memcpy(p.init_u_mean, cfg->init_u_mean_mv, sizeof(p.init_u_mean));
    std::memcpy(p.init_u_sd, cfg->init_u_sd_mv, sizeof(p.init_u_sd));
    std::memcpy(p.init_i_mean, cfg->init_i_mean_pa, sizeof(p.init_i_mean));
    std::memcpy(p.init_i_sd, cfg->init_i_sd_pa, sizeof(p.init_i_sd));
    if (p.init_mode == 2)
        for (int a = 0; a < mc::kPops; ++a)
            if (!(p.init_u_sd[a] > 0.0) || !(p.init_u_mean[a] < cfg->theta_mv) || !(p.init_i_sd[a] >= 0.0))
                return fail(MC_ERR_ARG, "relaxed start needs sd_u > 0, mean_u < theta and sd_I >= 0 for every population");
    const double ref = p.t_ref_ms / p.dt_ms;
    if (!(ref >= 0.0 && ref < 255.0)) return fail(MC_ERR_ARG, "refractory time must be below 255 steps");
    return MC_OK;
}

// Allocate and fill the device store.  With `segs`, the synapses are drawn and
// sorted on the GPU (the host holds only the plan), and the host gets the row
// pointers and the ring depth back.
int upload(mc_net *nt, const mc_config *cfg, const std::vector<mc::SynSeg> *segs)
{
    mc::HostNet &H = nt->host;
    const int64_t N = H.n, M = H.m;
    int rc;
    HIP_TRY(hipGetDevice(&nt->device));
    if ((rc = device_staging(nt->device, &nt->noalloc_ids))) return rc;
    {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, nt->device));
        nt->n_cu = prop.multiProcessorCount;
        nt->lds_limit = prop.sharedMemPerBlock;
    }
    HIP_TRY(hipStreamCreateWithFlags(&nt->stream, hipStreamNonBlocking));
    nt->own_stream = true;
    HIP_TRY(hipEventCreate(&nt->ev0));
    HIP_TRY(hipEventCreate(&nt->ev1));
    HIP_TRY(hipStreamCreateWithFlags(&nt->copy_stream, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipEventCreate(&nt->seg_ev0[b]));
        HIP_TRY(hipEventCreate(&nt->seg_ev1[b]));
        HIP_TRY(hipEventCreateWithFlags(&nt->snap_ev[b], hipEventDisableTiming));
    }

    if ((rc = dalloc(&nt->row_ptr, N + 1)) || (rc = dalloc(&nt->tgt, M)) || (rc = dalloc(&nt->dly, M))) return rc;
    const size_t wbytes = nt->params.wfmt == mc::kWFp32 ? 4 : 2;
    {
        hipError_t e = hipMalloc(&nt->w, std::max<size_t>(1, M * wbytes));
        if (e != hipSuccess) return fail(MC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    if (segs) {
        int max_d = 1;
        int64_t max_in_abs = 0;
        std::string msg;
        rc = mc::build_synapses_on_device(nt->params, H, *segs, nt->row_ptr, nt->tgt, nt->dly, nt->w, nt->stream, max_d,
                                          max_in_abs, msg);
        if (rc) return fail(rc, msg);
        if (max_in_abs + static_cast<int64_t>(mc::kPoisMax) * std::llabs(static_cast<long long>(nt->sc.wq_ext)) >=
            (int64_t{1} << 31))
            return fail(MC_ERR_OVERFLOW_BOUND, "int32 input-buffer overflow bound exceeded");
        H.ring = 2;
        while (H.ring < max_d + 1) H.ring *= 2;
        H.row_ptr.resize(static_cast<size_t>(N) + 1);
        HIP_TRY(hipMemcpy(H.row_ptr.data(), nt->row_ptr, (N + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
    }
    if ((rc = dalloc(&nt->u, N)) || (rc = dalloc(&nt->cur, N)) || (rc = dalloc(&nt->refr, N)) ||
        (rc = dalloc(&nt->meta, N)) || (rc = dalloc(&nt->inst_off, H.n_inst + 1)) ||
        (rc = dalloc(&nt->seeds, H.n_inst)) || (rc = dalloc(&nt->cdc, mc::kPops)) ||
        (rc = dalloc(&nt->pois_thr, mc::kPops * mc::kPoisMax)) ||
        (rc = dalloc(&nt->ring, static_cast<size_t>(H.ring) * N)) || (rc = dalloc(&nt->ctl, 1)))
        return rc;
    const int64_t work_cap = N + (M + 63) / 64 + 1;
    if ((rc = dalloc(&nt->work, work_cap))) return rc;
    nt->pois_slots = (N + 63) / 64 + 1;
    if ((rc = dalloc(&nt->pois_acc, nt->pois_slots))) return rc;
    int64_t cap = cfg->record_capacity;
    if (cap <= 0) cap = std::max<int64_t>(int64_t{1} << 22, 64 * N);
    nt->rec_cap = cap;
    for (int b = 0; b < 2; ++b) {
        const size_t bytes = sizeof(mc::RecHead) + static_cast<size_t>(cap) * sizeof(uint64_t);
        hipError_t e = hipMalloc(&nt->rblk[b], bytes);
        if (e != hipSuccess) return fail(MC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        HIP_TRY(hipHostMalloc(&nt->h_rblk[b], bytes, hipHostMallocDefault));
        // touched once here: the host's first access to a page of pinned memory
        // faults it in (~60 us for the head's page in a first run)
        std::memset(nt->h_rblk[b], 0, bytes);
        HIP_TRY(hipMemset(nt->rblk[b], 0, sizeof(mc::RecHead)));
        nt->rec[b] = reinterpret_cast<uint64_t *>(static_cast<char *>(nt->rblk[b]) + sizeof(mc::RecHead));
        nt->h_rec[b] = reinterpret_cast<uint64_t *>(static_cast<char *>(nt->h_rblk[b]) + sizeof(mc::RecHead));
        HIP_TRY(hipHostGetDevicePointer(&nt->hd_rblk[b], nt->h_rblk[b], 0));
    }
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&nt->h_ctl), sizeof(mc::StepCtl), hipHostMallocDefault));
    std::memset(nt->h_ctl, 0, sizeof(mc::StepCtl));

    // Static data.
    HIP_TRY(hipMemcpy(nt->meta, H.meta.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->inst_off, H.inst_off.data(), (H.n_inst + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->seeds, H.seeds.data(), H.n_inst * sizeof(uint64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->cdc, nt->sc.cdc, sizeof(nt->sc.cdc), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->pois_thr, nt->sc.pois_thr, sizeof(nt->sc.pois_thr), hipMemcpyHostToDevice));
    if (!segs) HIP_TRY(hipMemcpy(nt->row_ptr, H.row_ptr.data(), (N + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
    if (M && !segs) {
        HIP_TRY(hipMemcpy(nt->tgt, H.tgt.data(), M * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(nt->dly, H.d.data(), M, hipMemcpyHostToDevice));
        if (nt->params.wfmt == mc::kWFp32) {
            // float holding the fixed-point weight wq / 256 (exact for |wq| < 2^24)
            const int64_t chunk = int64_t{1} << 24;
            std::vector<float> tmp(static_cast<size_t>(std::min(M, chunk)));
            for (int64_t s0 = 0; s0 < M; s0 += chunk) {
                const int64_t s1 = std::min(M, s0 + chunk);
                for (int64_t s = s0; s < s1; ++s) tmp[s - s0] = static_cast<float>(H.wq[s]) * 0.00390625f;
                HIP_TRY(hipMemcpy(static_cast<float *>(nt->w) + s0, tmp.data(), (s1 - s0) * sizeof(float), hipMemcpyHostToDevice));
            }
        } else {
            HIP_TRY(hipMemcpy(nt->w, H.w16.data(), M * sizeof(uint16_t), hipMemcpyHostToDevice));
        }
    }
    // Dynamic state.
    HIP_TRY(hipMemcpy(nt->u, H.u0.data(), N * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->cur, H.i0.data(), N * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(nt->refr, 0, N));
    HIP_TRY(hipMemset(nt->ring, 0, static_cast<size_t>(H.ring) * N * sizeof(int32_t)));
    HIP_TRY(hipMemset(nt->ctl, 0, sizeof(mc::StepCtl)));
    HIP_TRY(hipMemset(nt->pois_acc, 0, nt->pois_slots * sizeof(unsigned long long)));
    HIP_TRY(hipDeviceSynchronize());
    return MC_OK;
}

// Cut every instance into tiles of at most `target` neurons (ceil(N_j/target)
// equal tiles); tiles never straddle instances.
void plan_tiles(const mc_net *nt, int target, std::vector<mc::TileDesc> &tiles, std::vector<int64_t> &sub_base,
                int64_t &sub_total, int &tile_max, int &max_intiles)
{
    tiles.clear();
    sub_base.assign(nt->host.n_inst, 0);
    sub_total = 0;
    tile_max = 0;
    max_intiles = 0;
    for (int j = 0; j < nt->host.n_inst; ++j) {
        const int32_t n0 = nt->host.inst_off[j], nn = nt->host.inst_off[j + 1] - n0;
        const int32_t T = (nn + target - 1) / target;
        const int32_t len = (nn + T - 1) / T;
        sub_base[j] = sub_total;
        const int32_t first = static_cast<int32_t>(tiles.size());
        for (int32_t k = 0; k < T; ++k) {
            mc::TileDesc d{};
            d.t0 = n0 + k * len;
            d.len = std::min(len, n0 + nn - d.t0);
            d.itile0 = first;
            d.intiles = T;
            d.inst_n0 = n0;
            d.stride = len;
            d.sub_base = sub_total + k;          // entry of (presynaptic p, tile k): sub_base + p * T
            tiles.push_back(d);
            tile_max = std::max(tile_max, d.len);
        }
        sub_total += static_cast<int64_t>(nn) * T;
        max_intiles = std::max<int>(max_intiles, T);
    }
}

// Prepare the tiled engine for tiles of at most `target` neurons, the ring in
// LDS (ring_mode 1), in global memory (2) or in LDS when it fits (0): check that
// every workgroup can be resident at once, then build the per-instance sub-row
// pointers on the device.
int setup_tiled(mc_net *nt, int target, int ring_mode)
{
    if (target < 16 || target > 4096) return fail(MC_ERR_ARG, "tile must be in [16, 4096]");
    if (nt->host.m >= (int64_t{1} << 32)) return fail(MC_ERR_UNSUPPORTED, "tiled engine needs fewer than 2^32 synapses");
    std::vector<mc::TileDesc> tiles;
    std::vector<int64_t> sub_base;
    int64_t sub_total = 0;
    int tile_max = 0, max_intiles = 0;
    plan_tiles(nt, target, tiles, sub_base, sub_total, tile_max, max_intiles);
    const int T = static_cast<int>(tiles.size());
    const size_t lds_static = 8 * mc::kPoisMaxDev * sizeof(uint64_t) + 32 * sizeof(int);
    // packed record format: 4-byte records for 16-bit weights when the local
    // target and delay fit 10 and 6 bits
    int sf = mc::kSyn8F32;
    if (nt->params.wfmt != mc::kWFp32) {
        const bool compact = tile_max <= 1024 && nt->host.ring <= 64;
        if (nt->params.wfmt == mc::kWFp16) sf = compact ? mc::kSyn4F16 : mc::kSyn8F16;
        else sf = compact ? mc::kSyn4BF16 : mc::kSyn8BF16;
    }
    mc::TiledShape sh = mc::tiled_shape(tile_max, max_intiles, nt->host.ring, ring_mode != 2);
    if (sh.lds + lds_static > 160 * 1024) {
        if (ring_mode == 1) return fail(MC_ERR_UNSUPPORTED, "tile ring does not fit in LDS");
        sh = mc::tiled_shape(tile_max, max_intiles, nt->host.ring, false);
        if (sh.lds + lds_static > 160 * 1024) return fail(MC_ERR_UNSUPPORTED, "tile scratch does not fit in LDS");
    }
    if (!sh.lds_ring) {
        // the LDS left over holds a window of the nearest slots (delays up to win)
        const size_t used = lds_static + sh.lds + 8;
        const size_t room = used < 160 * 1024 ? 160 * 1024 - used : 0;
        const int win = static_cast<int>(std::min<size_t>(nt->host.ring - 1, room / (4 * static_cast<size_t>(tile_max))));
        sh = mc::tiled_shape(tile_max, max_intiles, nt->host.ring, false, win);
    }
    int per_cu = 0;
    HIP_TRY(mc::tiled_max_coresident(sf, sh, &per_cu));
    if (static_cast<int64_t>(per_cu) * nt->n_cu < T)
        return fail(MC_ERR_UNSUPPORTED, "tiles cannot all be resident at once (" + std::to_string(T) + " tiles)");
    if (nt->tile == target && nt->tiled_shape.lds_ring == sh.lds_ring && nt->subrow) return MC_OK;
    HIP_TRY(hipStreamSynchronize(nt->stream));
    for (void *b : {static_cast<void *>(nt->subrow), static_cast<void *>(nt->syn), static_cast<void *>(nt->xchg),
                    static_cast<void *>(nt->xent), static_cast<void *>(nt->dropped), static_cast<void *>(nt->abort_word),
                    static_cast<void *>(nt->tiles_dev), static_cast<void *>(nt->gring)})
        if (b) hipFree(b);
    if (nt->h_dropped) hipHostFree(nt->h_dropped);
    nt->h_dropped = nullptr;
    nt->dropped = nullptr;
    nt->abort_word = nullptr;
    nt->gring = nullptr;
    nt->gstride = 0;
    nt->subrow = nullptr;
    nt->syn = nullptr;
    nt->xchg = nullptr;
    nt->xent = nullptr;
    nt->tiles_dev = nullptr;
    nt->tile = 0;
    nt->exch_dirty = true;
    int rc;
    if ((rc = dalloc(&nt->subrow, static_cast<size_t>(sub_total))) || (rc = dalloc(&nt->xchg, 2 * T)) ||
        (rc = dalloc(&nt->xent, static_cast<size_t>(2) * T * tile_max)) || (rc = dalloc(&nt->tiles_dev, T)))
        return rc;
    if (!nt->paths) {
        if ((rc = dalloc(&nt->paths, mc::kPaths))) return rc;
        HIP_TRY(hipMemset(nt->paths, 0, mc::kPaths * sizeof(unsigned long long)));
    }
    if ((rc = dalloc(&nt->dropped, 2 * static_cast<size_t>(T))) || (rc = dalloc(&nt->abort_word, 1))) return rc;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&nt->h_dropped), 2 * static_cast<size_t>(T) * sizeof(unsigned long long),
                          hipHostMallocDefault));
    std::memset(nt->h_dropped, 0, 2 * static_cast<size_t>(T) * sizeof(unsigned long long));
    if (!sh.lds_ring) {
        nt->gstride = ((tile_max + 31) / 32) * 32;
        if ((rc = dalloc(&nt->gring, static_cast<size_t>(T) * nt->host.ring * nt->gstride))) return rc;
    }
    HIP_TRY(hipMemcpy(nt->tiles_dev, tiles.data(), T * sizeof(mc::TileDesc), hipMemcpyHostToDevice));
    HIP_TRY(hipMemsetAsync(nt->xent, 0, static_cast<size_t>(2) * T * tile_max * sizeof(uint64_t), nt->stream));
    nt->xent_high = 0;
    {
        const size_t rec = sf <= mc::kSyn8BF16 ? 8 : 4;
        // a whole number of 16-byte chunks, at least one: the injection reads the
        // store in aligned 16-byte chunks, idle lanes reading the first
        const size_t bytes = std::max<size_t>(16, (static_cast<size_t>(nt->host.m) * rec + 15) / 16 * 16);
        hipError_t e = hipMalloc(&nt->syn, bytes);
        if (e != hipSuccess) return fail(MC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    const mc::DevNet d = dev_view(nt);
    HIP_TRY(mc::launch_subrows(d, nt->tiles_dev, T, nt->host.n, nt->subrow, nt->stream));
    {
        std::vector<int32_t> tile_of(static_cast<size_t>(nt->host.n));
        for (int k = 0; k < T; ++k)
            for (int32_t q = 0; q < tiles[k].len; ++q) tile_of[tiles[k].t0 + q] = k;
        int32_t *tile_of_dev = nullptr;
        if ((rc = dalloc(&tile_of_dev, tile_of.size()))) return rc;
        hipError_t e = hipMemcpy(tile_of_dev, tile_of.data(), tile_of.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = mc::launch_pack_synapses(d, nt->tiles_dev, tile_of_dev, nt->host.m, sf, nt->syn, nt->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(nt->stream);
        hipFree(tile_of_dev);
        if (e != hipSuccess) return fail(MC_ERR_HIP, std::string("tiled store build: ") + hipGetErrorString(e));
    }
    nt->syn_fmt = sf;
    // lanes per spike for cursor delivery: half the mean sub-row length (two or
    // more records per lane keep more loads in flight; measured at full scale:
    // 8 lanes deliver 16 % more events per second than 16, 2x more than 32)
    if (!nt->lanes_set) {
        const int64_t mean_len = (nt->host.m + std::max<int64_t>(1, sub_total) - 1) / std::max<int64_t>(1, sub_total);
        nt->lanes = static_cast<int>(std::min<int64_t>(64, std::max<int64_t>(4, (mean_len + 1) / 2)));
    }
    nt->tile = target;
    nt->tiles_host = tiles;
    nt->n_tiles = T;
    nt->tile_max = tile_max;
    nt->max_intiles = max_intiles;
    if (!nt->poll_delay_set) nt->poll_delay = max_intiles >= kPollDelayTiles ? kPollDelayDefault : 0;
    nt->tiled_shape = sh;
    return MC_OK;
}

// Smallest tile size >= `start` for which the instances need at most `cap` tiles
// (each instance rounds its tile count up).
int64_t fitting_tile(const mc_net *nt, int64_t cap, int64_t start)
{
    for (int64_t target = start; target <= 4096; target += std::max<int64_t>(1, target / 64)) {
        int64_t tiles = 0;
        for (int j = 0; j < nt->host.n_inst; ++j) {
            const int64_t nn = nt->host.inst_off[j + 1] - nt->host.inst_off[j];
            tiles += (nn + target - 1) / target;
        }
        if (tiles <= cap) return target;
    }
    return 4097;
}

// Default tiling: the ring in LDS with 1..4 workgroups per compute unit when it
// fits; otherwise a global-memory ring with 2, 1, 3 or 4 workgroups per CU.
int setup_tiled_default(mc_net *nt)
{
    const int64_t N = nt->host.n;
    const int64_t cus = nt->n_cu > 0 ? nt->n_cu : 256;
    for (int mode : {1, 2}) {
        for (int per_cu : mode == 1 ? std::vector<int>{1, 2, 3, 4} : std::vector<int>{2, 1, 3, 4}) {
            const int64_t target = fitting_tile(nt, cus * per_cu, std::max<int64_t>(64, (N + cus * per_cu - 1) / (cus * per_cu)));
            if (target > 4096) continue;
            if (setup_tiled(nt, static_cast<int>(target), mode) == MC_OK) return MC_OK;
        }
    }
    return fail(MC_ERR_UNSUPPORTED, "no tiling of this network fits the GPU");
}

int build_common(const uint64_t *seeds, const double *scales, int32_t n, const mc_config *cfg, mc_net **out)
{
    if (!out) return fail(MC_ERR_ARG, "out must not be NULL");
    *out = nullptr;
    if (!seeds || !scales || n < 1) return fail(MC_ERR_ARG, "need at least one (seed, scale)");
    mc_net *nt = new (std::nothrow) mc_net();
    if (!nt) return fail(MC_ERR_NOMEM, "out of host memory");
    int rc = params_from_config(cfg, nt->params);
    if (rc) { release(nt); return rc; }
    mc::derive_constants(nt->params, nt->sc);
    std::string msg;
    std::vector<mc::SynSeg> segs;
    try {
        rc = cfg->device_build ? mc::plan_network(nt->params, seeds, scales, n, nt->host, segs, msg)
                               : mc::build_host_network(nt->params, seeds, scales, n, nt->host, msg);
    } catch (const std::bad_alloc &) {
        rc = MC_ERR_NOMEM;
        msg = "out of host memory";
    } catch (...) {
        rc = MC_ERR_ARG;
        msg = "network build failed";
    }
    if (rc) { release(nt); return fail(rc, msg); }
    rc = upload(nt, cfg, cfg->device_build ? &segs : nullptr);
    if (rc) { release(nt); return rc; }
    // Keep only what the host needs after upload.
    std::vector<int32_t>().swap(nt->host.tgt);
    std::vector<int32_t>().swap(nt->host.wq);
    std::vector<uint16_t>().swap(nt->host.w16);
    std::vector<uint8_t>().swap(nt->host.d);
    nt->unread.assign(n, {});
    nt->counted.assign(n, 0);
    // capacity for the spikes of a few hundred steps, its pages touched now
    // rather than by the first run that records that many
    for (auto &v : nt->unread) {
        v.resize(std::max<size_t>(1024, kUnreadPrefault / static_cast<size_t>(n)));
        v.clear();
    }
    nt->inst_spikes.assign(n, 0);
    nt->inst_events.assign(n, 0);
    nt->inst_dropped.assign(n, 0);
    nt->inst_max_step.assign(n, 0);
    nt->engine = MC_ENGINE_GRAPH;
    if (cfg->engine != MC_ENGINE_GRAPH) {
        rc = setup_tiled_default(nt);
        if (rc == MC_OK) {
            nt->engine = MC_ENGINE_TILED;
        } else if (cfg->engine == MC_ENGINE_TILED) {
            release(nt);
            return rc;
        }
    }
    g_err.clear();
    *out = nt;
    return MC_OK;
}


// Add the out-degrees of the recorded spikes not yet counted to their
// instances' event counts.  A short run leaves this to the calls that read the
// counters, the spikes or a snapshot: it reads the row pointers at random
// places, which a run of a few steps would otherwise pay for from a cold cache.
void settle_events(mc_net *nt)
{
    const auto &rp = nt->host.row_ptr;
    for (int j = 0; j < nt->host.n_inst; ++j) {
        const auto &v = nt->unread[static_cast<size_t>(j)];
        const int64_t off = nt->host.inst_off[j];
        int64_t ev = 0;
        for (size_t q = nt->counted[static_cast<size_t>(j)]; q < v.size(); ++q) {
            const int64_t gid = off + v[q].second;
            ev += static_cast<int64_t>(rp[gid + 1] - rp[gid]);
        }
        nt->inst_events[static_cast<size_t>(j)] += ev;
        nt->counted[static_cast<size_t>(j)] = v.size();
    }
}

// Fold the spikes of the steps [s0, s0 + span) that a recorder holds (`total`
// recorded, `flags` of the launch, host copy `recs`) into the per-instance
// record and counters, and check the error flags.
int absorb(mc_net *nt, int64_t total, uint32_t flags, const uint64_t *recs, int64_t s0, int64_t span)
{
    if (flags & mc::kFlagTimeout) return fail(MC_ERR_HIP, "a cross-tile wait timed out");
    const int64_t got = std::min(total, nt->rec_cap);
    const auto &rp = nt->host.row_ptr;
    const auto &meta = nt->host.meta;
    const int n_inst = nt->host.n_inst;
    span = std::max<int64_t>(1, span);
    if (got < kAbsorbSerial) {
        // A short record (a short run, or a segment at a low rate): one pass on
        // this thread, each spike appended to its instance's list, with the
        // per-step counts in scratch kept across calls.
        std::vector<int32_t> &per = nt->absorb_scratch;
        per.assign(static_cast<size_t>(span) * n_inst, 0);
        for (int64_t q = 0; q < got; ++q) {
            const int32_t gid = static_cast<int32_t>(static_cast<uint32_t>(recs[q]));
            const int inst = n_inst == 1 ? 0 : static_cast<int>(meta[gid] >> 3);
            const int64_t n = static_cast<int64_t>(recs[q] >> 32);
            nt->unread[inst].emplace_back(n, gid - nt->host.inst_off[inst]);
            nt->inst_spikes[inst] += 1;
            const int64_t k = n - s0;
            if (k >= 0 && k < span) per[static_cast<size_t>(k) * n_inst + inst] += 1;
        }
        for (int64_t k = 0; k < span; ++k) {
            int64_t step_total = 0;
            for (int j = 0; j < n_inst; ++j) {
                const int64_t c = per[static_cast<size_t>(k) * n_inst + j];
                step_total += c;
                nt->inst_max_step[j] = std::max(nt->inst_max_step[j], c);
            }
            nt->max_step_spikes = std::max(nt->max_step_spikes, step_total);
        }
        if (total > nt->rec_cap || (flags & mc::kFlagRecordOverflow)) nt->overflow = true;
        return MC_OK;
    }
    // Threads take contiguous chunks of the record: a first pass counts spikes,
    // events and per-step spikes per instance, a second writes each spike into
    // its instance's list at the offset the counts give (order within a list
    // does not matter: mc_get_spikes sorts).
    const int nth = static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    struct Part {
        std::vector<int64_t> cnt, ev;
        std::vector<int32_t> per_step, per_inst_step;
    };
    std::vector<Part> part(static_cast<size_t>(nth));
    auto chunk = [got, nth](int t, int64_t &q0, int64_t &q1) {
        q0 = got * t / nth;
        q1 = got * (t + 1) / nth;
    };
    auto count = [&](int t) {
        Part &P = part[static_cast<size_t>(t)];
        P.cnt.assign(n_inst, 0);
        P.ev.assign(n_inst, 0);
        P.per_step.assign(static_cast<size_t>(span), 0);
        if (n_inst > 1) P.per_inst_step.assign(static_cast<size_t>(span) * n_inst, 0);
        int64_t q0, q1;
        chunk(t, q0, q1);
        for (int64_t q = q0; q < q1; ++q) {
            const int32_t gid = static_cast<int32_t>(static_cast<uint32_t>(recs[q]));
            const int inst = static_cast<int>(meta[gid] >> 3);
            P.cnt[inst] += 1;
            P.ev[inst] += static_cast<int64_t>(rp[gid + 1] - rp[gid]);
            const int64_t k = static_cast<int64_t>(recs[q] >> 32) - s0;
            if (k >= 0 && k < span) {
                P.per_step[k] += 1;
                if (n_inst > 1) P.per_inst_step[static_cast<size_t>(k) * n_inst + inst] += 1;
            }
        }
    };
    std::vector<std::vector<int64_t>> at(static_cast<size_t>(nth), std::vector<int64_t>(n_inst));
    auto place = [&](int t) {
        std::vector<int64_t> &cur = at[static_cast<size_t>(t)];
        int64_t q0, q1;
        chunk(t, q0, q1);
        for (int64_t q = q0; q < q1; ++q) {
            const int32_t gid = static_cast<int32_t>(static_cast<uint32_t>(recs[q]));
            const int inst = static_cast<int>(meta[gid] >> 3);
            nt->unread[inst][static_cast<size_t>(cur[inst]++)] = {static_cast<int64_t>(recs[q] >> 32),
                                                                  gid - nt->host.inst_off[inst]};
        }
    };
    auto parallel = [nth](auto &&f) {
        if (nth == 1) {
            f(0);
            return;
        }
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; ++t) pool.emplace_back(f, t);
        f(0);
        for (auto &th : pool) th.join();
    };
    settle_events(nt);
    parallel(count);
    for (int j = 0; j < n_inst; ++j) {
        int64_t off = static_cast<int64_t>(nt->unread[j].size());
        for (int t = 0; t < nth; ++t) {
            at[static_cast<size_t>(t)][j] = off;
            off += part[static_cast<size_t>(t)].cnt[j];
            nt->inst_spikes[j] += part[static_cast<size_t>(t)].cnt[j];
            nt->inst_events[j] += part[static_cast<size_t>(t)].ev[j];
        }
        nt->unread[j].resize(static_cast<size_t>(off));
        nt->counted[j] = static_cast<size_t>(off);
    }
    parallel(place);
    std::vector<int32_t> &per_step = part[0].per_step, &per_inst_step = part[0].per_inst_step;
    for (int t = 1; t < nth; ++t) {
        for (int64_t k = 0; k < span; ++k) per_step[k] += part[static_cast<size_t>(t)].per_step[k];
        for (size_t k = 0; k < per_inst_step.size(); ++k) per_inst_step[k] += part[static_cast<size_t>(t)].per_inst_step[k];
    }
    for (int64_t k = 0; k < span; ++k) {
        nt->max_step_spikes = std::max<int64_t>(nt->max_step_spikes, per_step[k]);
        if (nt->host.n_inst == 1) nt->inst_max_step[0] = nt->max_step_spikes;
        else
            for (int j = 0; j < nt->host.n_inst; ++j)
                nt->inst_max_step[j] = std::max<int64_t>(nt->inst_max_step[j], per_inst_step[static_cast<size_t>(k) * nt->host.n_inst + j]);
    }
    if (total > nt->rec_cap || (flags & mc::kFlagRecordOverflow)) nt->overflow = true;
    return MC_OK;
}

// Copy the recorder to the host, reset it, fold it in (the serial form).
int drain(mc_net *nt)
{
    HIP_TRY(hipMemcpyAsync(nt->h_ctl, nt->ctl, sizeof(mc::StepCtl), hipMemcpyDeviceToHost, nt->stream));
    HIP_TRY(hipStreamSynchronize(nt->stream));
    const int64_t got = std::min(nt->h_ctl->rec_total, nt->rec_cap);
    if (got > 0)
        HIP_TRY(hipMemcpyAsync(nt->h_rec[0], nt->rec[0], got * sizeof(uint64_t), hipMemcpyDeviceToHost, nt->stream));
    HIP_TRY(hipMemsetAsync(&nt->ctl->rec_total, 0, sizeof(int64_t), nt->stream));
    HIP_TRY(hipMemsetAsync(&nt->ctl->flags, 0, sizeof(uint32_t), nt->stream));
    HIP_TRY(hipStreamSynchronize(nt->stream));
    return absorb(nt, nt->h_ctl->rec_total, nt->h_ctl->flags, nt->h_rec[0], nt->step, nt->steps_in_flight);
}

// Steps until the next drain: keep the recorder at most a quarter full at the
// spike rate of the last segment.
void adapt_segment(mc_net *nt, int64_t steps_done, int64_t spikes_done)
{
    const double per_step = steps_done > 0 ? static_cast<double>(spikes_done) / steps_done : 0.0;
    const double fit = static_cast<double>(nt->rec_cap) / (4.0 * per_step + 64.0);
    nt->seg_steps = std::max<int64_t>(kSegMin, std::min<int64_t>(kSegMax, static_cast<int64_t>(fit)));
}

int run_tiled(mc_net *nt, int64_t steps)
{
    mc::TiledNet tn{};
    tn.base = dev_view(nt);
    tn.n_tiles = nt->n_tiles;
    tn.tile_max = nt->tile_max;
    tn.max_intiles = nt->max_intiles;
    tn.tiles = nt->tiles_dev;
    tn.gring = nt->gring;
    tn.gstride = nt->gstride;
    tn.subrow = nt->subrow;
    tn.syn = nt->syn;
    tn.syn_fmt = nt->syn_fmt;
    tn.xchg = nt->xchg;
    tn.poll_delay = nt->poll_delay;
    tn.win = nt->tiled_shape.win;
    tn.xent = nt->xent;
    tn.abort_word = nt->abort_word;
    tn.spin_limit = nt->spin_limit;
    tn.paths = nt->paths;
    tn.lanes = nt->lanes;
    const int T = nt->n_tiles;
    // Clearing is needed only in rare cases: entry words (tagged with their
    // step) and tile words (tagged with the step mod 32767) after the step index
    // went back (checkpoint load, tuner roll-back), tile words also after a jump
    // ahead far enough for an old tag to come round again, and the per-launch
    // counters after a new tiling, a checkpoint load or a failure.  A launch
    // otherwise starts with no host-side clearing at all.
    if (nt->step < nt->xent_high)
        HIP_TRY(hipMemsetAsync(nt->xent, 0, static_cast<size_t>(2) * T * nt->tile_max * sizeof(uint64_t), nt->stream));
    if (nt->exch_dirty || nt->step < nt->xchg_high || nt->step - nt->xchg_high > kTagSafe)
        HIP_TRY(hipMemsetAsync(nt->xchg, 0, 2 * static_cast<size_t>(T) * sizeof(uint64_t), nt->stream));
    if (nt->exch_dirty) {
        for (void *b : nt->rblk) HIP_TRY(hipMemsetAsync(b, 0, sizeof(mc::RecHead), nt->stream));
        HIP_TRY(hipMemsetAsync(nt->abort_word, 0, sizeof(uint32_t), nt->stream));
    }
    nt->exch_dirty = false;
    // Segments alternate between the two recorders.  After enqueueing segment k
    // (kernel, then copies of its counters and of the first part of its
    // recorder into pinned memory) the host folds in segment k-1 while segment k
    // runs; the recorder copy is sized from the last spike rate, and only a
    // segment that recorded more needs a second copy.
    struct Pending {
        int64_t s0, len, copied;
        int buf;
        bool budget;
    };
    Pending pend{0, 0, 0, -1, false};
    const bool timing = nt->timing;
    auto finish = [nt, timing, T](const Pending &p) -> int {
        HIP_TRY(hipEventSynchronize(nt->snap_ev[p.buf]));
        const mc::RecHead &c = *static_cast<const mc::RecHead *>(nt->h_rblk[p.buf]);
        if (timing) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, nt->seg_ev0[p.buf], nt->seg_ev1[p.buf]));
            nt->kernel_ms += ms;
            nt->launches += 1;
        }
        const int64_t total = static_cast<int64_t>(c.rec_total);
        const int64_t got = std::min(total, nt->rec_cap);
        if (got > p.copied && !(c.flags & mc::kFlagTimeout)) {
            HIP_TRY(hipMemcpyAsync(nt->h_rec[p.buf] + p.copied, nt->rec[p.buf] + p.copied,
                                   (got - p.copied) * sizeof(uint64_t), hipMemcpyDeviceToHost, nt->copy_stream));
            HIP_TRY(hipStreamSynchronize(nt->copy_stream));
        }
        if (p.budget) {
            const unsigned long long *dr = nt->h_dropped + static_cast<size_t>(p.buf) * T;
            for (int k = 0; k < T; ++k)
                if (dr[k]) nt->inst_dropped[nt->host.meta[nt->tiles_host[k].t0] >> 3] += static_cast<int64_t>(dr[k]);
        }
        const int64_t before = std::accumulate(nt->inst_spikes.begin(), nt->inst_spikes.end(), int64_t{0});
        const int rc = absorb(nt, total, c.flags, nt->h_rec[p.buf], p.s0, p.len);
        const int64_t after = std::accumulate(nt->inst_spikes.begin(), nt->inst_spikes.end(), int64_t{0});
        if (rc == MC_OK) {
            nt->rec_rate = static_cast<double>(after - before) / std::max<int64_t>(1, p.len);
            adapt_segment(nt, p.len, after - before);
        }
        return rc;
    };
    bool first = true;
    int rc = MC_OK;
    while (steps > 0 && rc == MC_OK) {
        // the phase trace covers the first steps of the first launch of this run
        tn.trace = first && nt->trace_tiles == T ? nt->trace : nullptr;
        tn.trace_steps = nt->trace_steps;
        first = false;
        const int64_t seg = std::min(steps, nt->seg_steps);
        const int b = nt->next_buf;
        if (++nt->epoch == 0) nt->epoch = 1;
        tn.head = static_cast<mc::RecHead *>(nt->rblk[b]);
        tn.head_other = static_cast<mc::RecHead *>(nt->rblk[b ^ 1]);
        tn.dropped = nt->dropped + static_cast<size_t>(b) * T;
        tn.epoch = nt->epoch;
        tn.base.rec = nt->rec[b];
        tn.budget_ticks = nt->budget_ticks;
        const int64_t guess = std::min<int64_t>(
            nt->rec_cap, 4096 + static_cast<int64_t>(static_cast<double>(seg) * std::max(64.0, 2.0 * nt->rec_rate)));
        if (timing) HIP_TRY(hipEventRecord(nt->seg_ev0[b], nt->stream));
        // An ordinary launch only while every workgroup has a compute unit of its
        // own: with several tiles per CU nothing but a cooperative launch makes
        // the runtime place them all at once, and a tile whose workgroup is not
        // placed would leave the others waiting for its words.
        const bool coop = nt->coop || (nt->n_cu > 0 && T > nt->n_cu);
        HIP_TRY(mc::launch_tiled(tn, nt->tiled_shape, seg, coop, nt->stream));
        if (timing) HIP_TRY(hipEventRecord(nt->seg_ev1[b], nt->stream));
        // the head and the first `guess` entries (at most as many as were
        // recorded), written into the pinned buffer by a kernel of ours: it
        // starts sooner after the step kernel than the runtime's copy does
        HIP_TRY(mc::launch_copy_out(static_cast<const mc::RecHead *>(nt->rblk[b]), nt->rec[b], guess,
                                    static_cast<mc::RecHead *>(nt->hd_rblk[b]),
                                    reinterpret_cast<uint64_t *>(static_cast<char *>(nt->hd_rblk[b]) + sizeof(mc::RecHead)),
                                    nt->stream));
        if (tn.budget_ticks)
            HIP_TRY(hipMemcpyAsync(nt->h_dropped + static_cast<size_t>(b) * T, tn.dropped, T * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, nt->stream));
        HIP_TRY(hipEventRecord(nt->snap_ev[b], nt->stream));
        nt->xent_high = std::max(nt->xent_high, nt->step + seg);
        nt->xchg_high = nt->step + seg;
        if (pend.buf >= 0) rc = finish(pend);
        pend = {nt->step, seg, guess, b, tn.budget_ticks != 0};
        nt->next_buf ^= 1;
        nt->step += seg;
        steps -= seg;
    }
    if (pend.buf >= 0) {
        if (rc == MC_OK) rc = finish(pend);
        else HIP_TRY(hipStreamSynchronize(nt->stream));
    }
    return rc;
}

int ensure_graph(mc_net *nt)
{
    if (nt->graph_exec && nt->graph_k == nt->graph_chunk) return MC_OK;
    if (nt->graph_exec) {
        hipGraphExecDestroy(nt->graph_exec);
        nt->graph_exec = nullptr;
    }
    const mc::DevNet d = dev_view(nt);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(nt->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < nt->graph_chunk && e == hipSuccess; ++s) {
        e = mc::launch_neuron(d, nt->block, s, nt->stream);
        if (e == hipSuccess) e = mc::launch_deliver(d, nt->deliver_grid, s, nt->stream);
    }
    if (e == hipSuccess) e = mc::launch_advance(d, nt->graph_chunk, nt->stream);
    hipError_t e2 = hipStreamEndCapture(nt->stream, &g);
    if (e != hipSuccess) { if (g) hipGraphDestroy(g); return fail(MC_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e)); }
    if (e2 != hipSuccess) return fail(MC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(&nt->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) { nt->graph_exec = nullptr; return fail(MC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); }
    nt->graph_k = nt->graph_chunk;
    return MC_OK;
}

int run_graph(mc_net *nt, int64_t steps)
{
    if (nt->budget_ticks) return fail(MC_ERR_UNSUPPORTED, "the step budget needs the tiled engine");
    int rc = ensure_graph(nt);
    if (rc) return rc;
    const mc::DevNet d = dev_view(nt);
    // The per-step counts are only meaningful inside a graph run; another engine
    // may have advanced the step index since, so start from clean buffers.
    HIP_TRY(hipMemsetAsync(nt->ctl->cnt, 0, sizeof(nt->ctl->cnt), nt->stream));
    while (steps > 0) {
        const int64_t seg = std::min(steps, nt->seg_steps);
        const int64_t chunks = seg / nt->graph_chunk;
        const int rem = static_cast<int>(seg % nt->graph_chunk);
        if (nt->timing) HIP_TRY(hipEventRecord(nt->ev0, nt->stream));
        for (int64_t c = 0; c < chunks; ++c) HIP_TRY(hipGraphLaunch(nt->graph_exec, nt->stream));
        for (int s = 0; s < rem; ++s) {
            HIP_TRY(mc::launch_neuron(d, nt->block, s, nt->stream));
            HIP_TRY(mc::launch_deliver(d, nt->deliver_grid, s, nt->stream));
        }
        if (rem) HIP_TRY(mc::launch_advance(d, rem, nt->stream));
        if (nt->timing) {
            HIP_TRY(hipEventRecord(nt->ev1, nt->stream));
            HIP_TRY(hipEventSynchronize(nt->ev1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, nt->ev0, nt->ev1));
            nt->kernel_ms += ms;
            nt->launches += seg;
        }
        const int64_t before = std::accumulate(nt->inst_spikes.begin(), nt->inst_spikes.end(), int64_t{0});
        nt->steps_in_flight = seg;
        if ((rc = drain(nt))) return rc;
        const int64_t after = std::accumulate(nt->inst_spikes.begin(), nt->inst_spikes.end(), int64_t{0});
        adapt_segment(nt, seg, after - before);
        nt->step += seg;
        steps -= seg;
    }
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Dynamic-state snapshots: device state (neuron state, rings, step control,
// Poisson counters) plus the host-side run state.  Used by the autotuner (trials
// run on a copy and are rolled back) and by checkpoint files.
// ---------------------------------------------------------------------------
struct Snapshot {
    std::vector<float> u, cur;
    std::vector<uint8_t> refr;
    std::vector<int32_t> ring;
    mc::StepCtl ctl{};
    std::vector<unsigned long long> pois;
    int64_t step = 0;
    std::vector<std::vector<std::pair<int64_t, int32_t>>> unread;
    std::vector<int64_t> inst_spikes, inst_events, inst_max_step, inst_dropped;
    int64_t max_step_spikes = 0;
};

int take_snapshot(mc_net *nt, Snapshot &s)
{
    const int64_t N = nt->host.n;
    s.u.resize(N);
    s.cur.resize(N);
    s.refr.resize(N);
    s.ring.resize(static_cast<size_t>(nt->host.ring) * N);
    s.pois.resize(nt->pois_slots);
    HIP_TRY(hipStreamSynchronize(nt->stream));
    HIP_TRY(hipMemcpy(s.u.data(), nt->u, N * sizeof(float), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(s.cur.data(), nt->cur, N * sizeof(float), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(s.refr.data(), nt->refr, N, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(s.ring.data(), nt->ring, s.ring.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&s.ctl, nt->ctl, sizeof(s.ctl), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(s.pois.data(), nt->pois_acc, s.pois.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    s.step = nt->step;
    settle_events(nt);
    s.unread = nt->unread;
    s.inst_spikes = nt->inst_spikes;
    s.inst_events = nt->inst_events;
    s.inst_dropped = nt->inst_dropped;
    s.inst_max_step = nt->inst_max_step;
    s.max_step_spikes = nt->max_step_spikes;
    return MC_OK;
}

int restore_snapshot(mc_net *nt, const Snapshot &s)
{
    const int64_t N = nt->host.n;
    HIP_TRY(hipStreamSynchronize(nt->stream));
    HIP_TRY(hipMemcpy(nt->u, s.u.data(), N * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->cur, s.cur.data(), N * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->refr, s.refr.data(), N, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->ring, s.ring.data(), s.ring.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->ctl, &s.ctl, sizeof(s.ctl), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(nt->pois_acc, s.pois.data(), s.pois.size() * sizeof(unsigned long long), hipMemcpyHostToDevice));
    nt->step = s.step;
    for (size_t j = 0; j < nt->unread.size(); ++j) {
        // element-wise, keeping each list's capacity (touched at build)
        nt->unread[j].assign(s.unread[j].begin(), s.unread[j].end());
        nt->counted[j] = nt->unread[j].size();
    }
    nt->inst_spikes = s.inst_spikes;
    nt->inst_events = s.inst_events;
    nt->inst_dropped = s.inst_dropped;
    nt->inst_max_step = s.inst_max_step;
    nt->max_step_spikes = s.max_step_spikes;
    nt->exch_dirty = true;            // tile words and counters of abandoned launches
    nt->failed = false;
    nt->fail_msg.clear();
    return MC_OK;
}

constexpr char kCkptMagic[8] = {'M', 'C', 'C', 'K', 'P', 'T', '0', '3'};

template <class T>
bool put(std::FILE *f, const T *p, size_t n) { return std::fwrite(p, sizeof(T), n, f) == n; }
template <class T>
bool get(std::FILE *f, T *p, size_t n) { return std::fread(p, sizeof(T), n, f) == n; }

int write_checkpoint(mc_net *nt, const char *path)
{
    Snapshot s;
    int rc = take_snapshot(nt, s);
    if (rc) return rc;
    std::FILE *f = std::fopen(path, "wb");
    if (!f) return fail(MC_ERR_IO, std::string("cannot open ") + path);
    const int64_t hdr[6] = {nt->host.n, nt->host.m, nt->host.ring, nt->host.n_inst, nt->params.wfmt,
                            static_cast<int64_t>(s.pois.size())};
    bool ok = put(f, kCkptMagic, 8) && put(f, hdr, 6) && put(f, nt->host.seeds.data(), nt->host.seeds.size()) &&
              put(f, nt->host.scales.data(), nt->host.scales.size()) && put(f, &s.step, 1) &&
              put(f, s.u.data(), s.u.size()) && put(f, s.cur.data(), s.cur.size()) &&
              put(f, s.refr.data(), s.refr.size()) && put(f, s.ring.data(), s.ring.size()) && put(f, &s.ctl, 1) &&
              put(f, s.pois.data(), s.pois.size()) && put(f, s.inst_spikes.data(), s.inst_spikes.size()) &&
              put(f, s.inst_events.data(), s.inst_events.size()) && put(f, s.inst_max_step.data(), s.inst_max_step.size()) &&
              put(f, s.inst_dropped.data(), s.inst_dropped.size()) &&
              put(f, &s.max_step_spikes, 1);
    for (const auto &v : s.unread) {
        const int64_t k = static_cast<int64_t>(v.size());
        ok = ok && put(f, &k, 1) && put(f, v.data(), v.size());
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? MC_OK : fail(MC_ERR_IO, std::string("write failed: ") + path);
}

int read_checkpoint(mc_net *nt, const char *path)
{
    std::FILE *f = std::fopen(path, "rb");
    if (!f) return fail(MC_ERR_IO, std::string("cannot open ") + path);
    char magic[8];
    int64_t hdr[6];
    Snapshot s;
    std::vector<uint64_t> seeds(nt->host.n_inst);
    std::vector<double> scales(nt->host.n_inst);
    bool ok = get(f, magic, 8) && std::memcmp(magic, kCkptMagic, 8) == 0 && get(f, hdr, 6);
    ok = ok && hdr[0] == nt->host.n && hdr[1] == nt->host.m && hdr[2] == nt->host.ring && hdr[3] == nt->host.n_inst &&
         hdr[4] == nt->params.wfmt && hdr[5] == nt->pois_slots;
    ok = ok && get(f, seeds.data(), seeds.size()) && get(f, scales.data(), scales.size()) &&
         seeds == nt->host.seeds && scales == nt->host.scales;
    if (!ok) {
        std::fclose(f);
        return fail(MC_ERR_ARG, "checkpoint does not belong to a network built with the same arguments");
    }
    const int64_t N = nt->host.n;
    s.u.resize(N);
    s.cur.resize(N);
    s.refr.resize(N);
    s.ring.resize(static_cast<size_t>(nt->host.ring) * N);
    s.pois.resize(nt->pois_slots);
    s.inst_spikes.resize(nt->host.n_inst);
    s.inst_events.resize(nt->host.n_inst);
    s.inst_max_step.resize(nt->host.n_inst);
    s.inst_dropped.resize(nt->host.n_inst);
    s.unread.resize(nt->host.n_inst);
    ok = get(f, &s.step, 1) && get(f, s.u.data(), N) && get(f, s.cur.data(), N) && get(f, s.refr.data(), N) &&
         get(f, s.ring.data(), s.ring.size()) && get(f, &s.ctl, 1) && get(f, s.pois.data(), s.pois.size()) &&
         get(f, s.inst_spikes.data(), s.inst_spikes.size()) && get(f, s.inst_events.data(), s.inst_events.size()) &&
         get(f, s.inst_max_step.data(), s.inst_max_step.size()) && get(f, s.inst_dropped.data(), s.inst_dropped.size()) &&
         get(f, &s.max_step_spikes, 1);
    for (auto &v : s.unread) {
        int64_t k = 0;
        ok = ok && get(f, &k, 1) && k >= 0 && k < (int64_t{1} << 40);
        if (!ok) break;
        v.resize(static_cast<size_t>(k));
        ok = get(f, v.data(), v.size());
    }
    std::fclose(f);
    if (!ok) return fail(MC_ERR_IO, std::string("truncated checkpoint: ") + path);
    return restore_snapshot(nt, s);
}

int run_engine(mc_net *nt, int64_t steps)
{
    return nt->engine == MC_ENGINE_TILED ? run_tiled(nt, steps) : run_graph(nt, steps);
}

// A launch configuration the tuner can select.
struct Candidate {
    int engine, tile, ring, graph_chunk, seg, block, grid;
    int poll;                         // tiled: poll delay, or -1 for the default of the tile count
};

int apply_candidate(mc_net *nt, const Candidate &c)
{
    if (c.engine == MC_ENGINE_TILED) {
        const int rc = setup_tiled(nt, c.tile, c.ring);
        if (rc) return rc;
        nt->engine = MC_ENGINE_TILED;
        nt->poll_delay_set = c.poll >= 0;
        nt->poll_delay = c.poll >= 0 ? c.poll : (nt->max_intiles >= kPollDelayTiles ? kPollDelayDefault : 0);
        return MC_OK;
    }
    if (nt->graph_chunk != c.graph_chunk || nt->seg != c.seg || nt->block != c.block || nt->deliver_grid != c.grid) {
        nt->graph_chunk = c.graph_chunk;
        nt->seg = c.seg;
        nt->block = c.block;
        nt->deliver_grid = c.grid;
        if (nt->graph_exec) {
            hipGraphExecDestroy(nt->graph_exec);
            nt->graph_exec = nullptr;
            nt->graph_k = 0;
        }
    }
    nt->engine = MC_ENGINE_GRAPH;
    return MC_OK;
}

// Time every candidate on the saved state, roll back after each trial, keep the
// fastest (the configuration in use unless another is clearly faster).  Every
// candidate computes bit-identical results, so the choice only changes speed.
int autotune(mc_net *nt, int64_t trial_steps)
{
    Snapshot s;
    int rc = take_snapshot(nt, s);
    if (rc) return rc;
    const bool timing = nt->timing;
    nt->timing = false;
    const int64_t seg_steps = nt->seg_steps;
    std::vector<Candidate> cands;
    const int64_t N = nt->host.n;
    const int cus = nt->n_cu > 0 ? nt->n_cu : 256;
    for (int ring : {1, 2})
        for (int per_cu : {1, 2, 3, 4}) {
            const int64_t cap = static_cast<int64_t>(cus) * per_cu;
            const int64_t tile = fitting_tile(nt, cap, std::max<int64_t>(64, (N + cap - 1) / cap));
            if (tile <= 4096) cands.push_back({MC_ENGINE_TILED, static_cast<int>(tile), ring, 0, 0, 0, 0, -1});
        }
    if (!nt->budget_ticks)            // the step budget needs the tiled engine
        for (int block : {128, 256, 512})
            for (int seg : {128, 256, 512})
                for (int grid : {512, 2048})
                    for (int chunk : {32, 128})
                        cands.push_back({MC_ENGINE_GRAPH, 0, 0, chunk, seg, block, grid, 0});
    double best = 1e300;
    Candidate pick{nt->engine, nt->tile, nt->tiled_shape.lds_ring ? 1 : 2, nt->graph_chunk, nt->seg, nt->block,
                   nt->deliver_grid, nt->poll_delay_set ? nt->poll_delay : -1};
    // Each candidate runs the same steps from the saved state twice; its time
    // is the faster of the two.  A candidate replaces the current pick only
    // when at least kTuneMargin faster: the trials are short, and a form that
    // wins one by a little can lose over a long run.
    auto trial = [&](const Candidate &c) -> int {
        if (apply_candidate(nt, c) != MC_OK) return MC_OK;   // e.g. the tile ring does not fit in LDS
        int r;
        if ((r = restore_snapshot(nt, s))) return r;
        nt->seg_steps = std::max<int64_t>(trial_steps, 1);
        if ((r = run_engine(nt, std::max<int64_t>(8, trial_steps / 8)))) return r;   // graph capture, warm caches
        double dt = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            if ((r = restore_snapshot(nt, s))) return r;
            const auto t0 = std::chrono::steady_clock::now();
            if ((r = run_engine(nt, trial_steps))) return r;
            dt = std::min(dt, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        }
        if (best >= 1e299 || dt < best * (1.0 - kTuneMargin)) {
            best = dt;
            pick = c;
        }
        return MC_OK;
    };
    const Candidate orig = pick;
    // A failed trial leaves the state inconsistent: go back to the launch
    // configuration and the state from before the tuner, then report.
    auto roll_back = [&](int code) {
        const std::string msg = g_err;
        apply_candidate(nt, orig);
        nt->seg_steps = seg_steps;
        nt->timing = timing;
        nt->overflow = false;
        if (restore_snapshot(nt, s) != MC_OK) {
            nt->failed = true;
            nt->fail_msg = msg;
        }
        g_err = msg;
        return code;
    };
    if ((rc = trial(orig))) return roll_back(rc);          // the configuration in use sets the bar
    for (const Candidate &c : cands)
        if ((rc = trial(c))) return roll_back(rc);
    // then the tiled engine's polling delay for the chosen tiles
    if (pick.engine == MC_ENGINE_TILED) {
        const Candidate base = pick;
        for (int d : {0, 8, 16, 24, 32, 48, 64}) {
            Candidate c = base;
            c.poll = d;
            if ((rc = trial(c))) return roll_back(rc);
        }
    }
    g_err.clear();
    if ((rc = apply_candidate(nt, pick))) return rc;
    nt->seg_steps = seg_steps;
    nt->timing = timing;
    nt->overflow = false;
    return restore_snapshot(nt, s);
}

// Checks shared by the two injection entry points (no allocation): instance,
// count and ids; *events = the synapses the listed rows hold.
int inject_check(mc_net *net, int32_t instance, const int32_t *ids, int64_t count, int64_t *events)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (instance < 0 || instance >= net->host.n_inst) return fail(MC_ERR_ARG, "instance out of range");
    LIVE_OR_FAIL(net);
    if (count < 0 || count > (int64_t{1} << 30)) return fail(MC_ERR_ARG, "count out of range");
    if (count > 0 && !ids) return fail(MC_ERR_ARG, "ids must not be NULL");
    const int32_t off = net->host.inst_off[instance];
    const int32_t nn = net->host.inst_off[instance + 1] - off;
    int64_t ev = 0;
    for (int64_t q = 0; q < count; ++q) {
        if (ids[q] < 0 || ids[q] >= nn) return fail(MC_ERR_ARG, "neuron id out of range");
        ev += static_cast<int64_t>(net->host.row_ptr[off + ids[q] + 1] - net->host.row_ptr[off + ids[q]]);
    }
    *events = ev;
    return MC_OK;
}

// Copy the instance-local ids into the device array `dev_ids` and deliver the
// listed rows (checked by inject_check).  Allocates nothing.
int inject_run(mc_net *net, int32_t instance, const int32_t *ids, int64_t count, int32_t *dev_ids)
{
    const int32_t off = net->host.inst_off[instance];
    HIP_TRY(hipMemcpyAsync(dev_ids, ids, count * sizeof(int32_t), hipMemcpyHostToDevice, net->stream));
    const mc::DevNet d = dev_view(net);
    if (net->timing) HIP_TRY(hipEventRecord(net->ev0, net->stream));
    if (net->engine == MC_ENGINE_TILED && mc::inject_batch(net->tile_max, net->host.ring) > 0) {
        mc::TiledNet tn{};
        tn.base = d;
        tn.n_tiles = net->n_tiles;
        tn.tile_max = net->tile_max;
        tn.tiles = net->tiles_dev;
        tn.subrow = net->subrow;
        tn.syn = net->syn;
        tn.syn_fmt = net->syn_fmt;
        tn.lanes = net->lanes;
        int first = 0;
        while (net->tiles_host[first].inst_n0 != off) ++first;
        const int threads = 1024;   // events, not neurons, spread over the threads: more loads in flight
        HIP_TRY(mc::launch_inject_tiled(tn, first, net->tiles_host[first].intiles, threads, dev_ids,
                                        static_cast<int32_t>(count), off, net->step, net->stream));
    } else {
        HIP_TRY(mc::launch_inject_global(d, dev_ids, static_cast<int32_t>(count), off, net->step, net->stream));
    }
    if (net->timing) {
        HIP_TRY(hipEventRecord(net->ev1, net->stream));
        HIP_TRY(hipEventSynchronize(net->ev1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, net->ev0, net->ev1));
        net->kernel_ms += ms;
        net->launches += 1;
    }
    HIP_TRY(hipStreamSynchronize(net->stream));
    return MC_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *mc_last_error(void) { return g_err.c_str(); }

int mc_config_default(mc_config *cfg)
{
    if (!cfg) return fail(MC_ERR_ARG, "cfg must not be NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(mc_config);
    cfg->conn_probs = nullptr;
    cfg->wfmt = MC_W_FP32;
    cfg->poisson_on = 1;
    cfg->init_mode = 0;
    cfg->engine = MC_ENGINE_AUTO;
    cfg->record_capacity = 0;
    const double full[MC_NPOP] = {20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948};
    const double kext[MC_NPOP] = {1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100};
    for (int a = 0; a < MC_NPOP; ++a) {
        cfg->full_size[a] = full[a];
        cfg->k_ext[a] = kext[a];
        cfg->i_dc_pa[a] = 0.0;
    }
    cfg->nu_bg_hz = 8.0;
    cfg->dt_ms = 0.1;
    cfg->tau_m_ms = 10.0;
    cfg->c_m_pf = 250.0;
    cfg->tau_syn_ms = 0.5;
    cfg->t_ref_ms = 2.0;
    cfg->theta_mv = 15.0;
    cfg->w_mean_pa = 87.8;
    cfg->w_sd_pa = 8.78;
    cfg->g = -4.0;
    cfg->l4e_l23e_factor = 2.0;
    cfg->w_ext_pa = 87.8;
    cfg->d_mean_exc_ms = 1.5;
    cfg->d_sd_exc_ms = 0.75;
    cfg->d_mean_inh_ms = 0.8;
    cfg->d_sd_inh_ms = 0.4;
    return MC_OK;
}

int mc_build_network(uint64_t seed, double scale, const mc_config *cfg, mc_net **out)
{
    return build_common(&seed, &scale, 1, cfg, out);
}

int mc_build_batch(const uint64_t *seeds, const double *scales, int32_t n, const mc_config *cfg, mc_net **out)
{
    return build_common(seeds, scales, n, cfg, out);
}

int mc_run(mc_net *net, int64_t steps)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    LIVE_OR_FAIL(net);
    if (steps < 0) return fail(MC_ERR_ARG, "steps must be >= 0");
    if (steps == 0) return MC_OK;
    if (net->step + steps >= (int64_t{1} << 31)) return fail(MC_ERR_ARG, "step index would exceed 2^31");
    int rc = net->engine == MC_ENGINE_TILED ? run_tiled(net, steps) : run_graph(net, steps);
    if (rc == MC_ERR_HIP) {
        net->failed = true;
        net->fail_msg = g_err;
    }
    if (rc) return rc;
    if (net->overflow) {
        net->overflow = false;
        return fail(MC_ERR_RECORD_OVERFLOW, "spike recorder overflowed; increase record_capacity");
    }
    return MC_OK;
}

int mc_get_spikes(mc_net *net, int32_t instance, int64_t *steps_out, int32_t *ids_out, int64_t cap, int64_t *count_out)
{
    if (!net || !count_out) return fail(MC_ERR_ARG, "net and count_out must not be NULL");
    LIVE_OR_FAIL(net);
    if (instance < 0 || instance >= net->host.n_inst) return fail(MC_ERR_ARG, "instance out of range");
    auto &v = net->unread[instance];
    *count_out = static_cast<int64_t>(v.size());
    if (cap < static_cast<int64_t>(v.size())) return fail(MC_ERR_BUFFER_TOO_SMALL, "buffer too small");
    if (!v.empty() && (!steps_out || !ids_out)) return fail(MC_ERR_ARG, "output buffers must not be NULL");
    settle_events(net);
    std::sort(v.begin(), v.end());
    for (size_t q = 0; q < v.size(); ++q) {
        steps_out[q] = v[q].first;
        ids_out[q] = v[q].second;
    }
    v.clear();
    net->counted[static_cast<size_t>(instance)] = 0;
    return MC_OK;
}

int mc_instance_size(mc_net *net, int32_t instance, int64_t *n_neurons, int64_t *n_synapses)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (instance < 0 || instance >= net->host.n_inst) return fail(MC_ERR_ARG, "instance out of range");
    if (n_neurons) *n_neurons = net->host.inst_off[instance + 1] - net->host.inst_off[instance];
    if (n_synapses) *n_synapses = net->host.inst_syn_off[instance + 1] - net->host.inst_syn_off[instance];
    return MC_OK;
}

int mc_get_state(mc_net *net, int32_t instance, float *u_mv, float *i_pa, int32_t *refr, int64_t n)
{
    int64_t nn = 0;
    int rc = mc_instance_size(net, instance, &nn, nullptr);
    if (rc) return rc;
    LIVE_OR_FAIL(net);
    if (n != nn) return fail(MC_ERR_ARG, "n must equal the instance's neuron count");
    const int64_t o = net->host.inst_off[instance];
    HIP_TRY(hipStreamSynchronize(net->stream));
    if (u_mv) HIP_TRY(hipMemcpy(u_mv, net->u + o, n * sizeof(float), hipMemcpyDeviceToHost));
    if (i_pa) HIP_TRY(hipMemcpy(i_pa, net->cur + o, n * sizeof(float), hipMemcpyDeviceToHost));
    if (refr) {
        std::vector<uint8_t> r(static_cast<size_t>(n));
        HIP_TRY(hipMemcpy(r.data(), net->refr + o, n, hipMemcpyDeviceToHost));
        for (int64_t q = 0; q < n; ++q) refr[q] = r[q];
    }
    return MC_OK;
}

int mc_set_state(mc_net *net, int32_t instance, const float *u_mv, const float *i_pa, const int32_t *refr, int64_t n)
{
    int64_t nn = 0;
    int rc = mc_instance_size(net, instance, &nn, nullptr);
    if (rc) return rc;
    LIVE_OR_FAIL(net);
    if (n != nn) return fail(MC_ERR_ARG, "n must equal the instance's neuron count");
    const int64_t o = net->host.inst_off[instance];
    HIP_TRY(hipStreamSynchronize(net->stream));
    if (u_mv) HIP_TRY(hipMemcpy(net->u + o, u_mv, n * sizeof(float), hipMemcpyHostToDevice));
    if (i_pa) HIP_TRY(hipMemcpy(net->cur + o, i_pa, n * sizeof(float), hipMemcpyHostToDevice));
    if (refr) {
        std::vector<uint8_t> r(static_cast<size_t>(n));
        for (int64_t q = 0; q < n; ++q) {
            if (refr[q] < 0 || refr[q] > 255) return fail(MC_ERR_ARG, "refractory count out of range");
            r[q] = static_cast<uint8_t>(refr[q]);
        }
        HIP_TRY(hipMemcpy(net->refr + o, r.data(), n, hipMemcpyHostToDevice));
    }
    return MC_OK;
}

int mc_get_counters(mc_net *net, int32_t instance, mc_counters *out)
{
    if (!net || !out) return fail(MC_ERR_ARG, "net and out must not be NULL");
    if (instance < -1 || instance >= net->host.n_inst) return fail(MC_ERR_ARG, "instance out of range");
    LIVE_OR_FAIL(net);
    std::vector<unsigned long long> acc(static_cast<size_t>(net->pois_slots));
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(hipMemcpy(acc.data(), net->pois_acc, acc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    settle_events(net);
    out->steps = net->step;
    out->spikes = 0;
    out->events = 0;
    out->dropped_events = 0;
    for (int j = 0; j < net->host.n_inst; ++j)
        if (instance < 0 || instance == j) {
            out->spikes += net->inst_spikes[j];
            out->events += net->inst_events[j];
            out->dropped_events += net->inst_dropped[j];
        }
    int64_t pe = 0;
    for (auto v : acc) pe += static_cast<int64_t>(v);
    out->poisson_events = pe;
    out->max_spikes_per_step = instance < 0 ? net->max_step_spikes : net->inst_max_step[instance];
    return MC_OK;
}

int mc_get_info(mc_net *net, mc_info *out)
{
    if (!net || !out) return fail(MC_ERR_ARG, "net and out must not be NULL");
    std::memset(out, 0, sizeof(*out));
    out->n_instances = net->host.n_inst;
    out->ring_depth = net->host.ring;
    out->engine = net->engine;
    out->wfmt = net->params.wfmt;
    out->n_neurons = net->host.n;
    out->n_synapses = net->host.m;
    out->tile_neurons = net->engine == MC_ENGINE_TILED ? net->tile_max : 0;
    out->lds_ring = net->engine == MC_ENGINE_TILED ? (net->tiled_shape.lds_ring ? 1 : 0) : 0;
    out->syn_bytes = net->engine == MC_ENGINE_TILED ? (net->syn_fmt <= mc::kSyn8BF16 ? 8 : 4)
                                                    : (net->params.wfmt == mc::kWFp32 ? 9 : 7);
    out->n_tiles = net->engine == MC_ENGINE_TILED ? net->n_tiles : 0;
    out->graph_chunk = net->graph_chunk;
    out->seg = net->seg;
    out->block = net->block;
    out->deliver_grid = net->deliver_grid;
    out->poll_delay = net->poll_delay;
    out->lds_window = net->engine == MC_ENGINE_TILED ? net->tiled_shape.win : 0;
    return MC_OK;
}

int mc_get_csr(mc_net *net, int32_t instance, int64_t *row_ptr, int32_t *post, int32_t *wq, uint8_t *d, int64_t n_synapses)
{
    int64_t nn = 0, mm = 0;
    int rc = mc_instance_size(net, instance, &nn, &mm);
    if (rc) return rc;
    if (n_synapses != mm) return fail(MC_ERR_ARG, "n_synapses must equal the instance's synapse count");
    LIVE_OR_FAIL(net);
    HIP_TRY(hipStreamSynchronize(net->stream));
    const int64_t o = net->host.inst_off[instance];
    const int64_t so = net->host.inst_syn_off[instance];
    if (row_ptr) {
        std::vector<uint64_t> rp(static_cast<size_t>(nn + 1));
        HIP_TRY(hipMemcpy(rp.data(), net->row_ptr + o, (nn + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
        for (int64_t q = 0; q <= nn; ++q) row_ptr[q] = static_cast<int64_t>(rp[q]) - so;
    }
    if (post) {
        HIP_TRY(hipMemcpy(post, net->tgt + so, mm * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t q = 0; q < mm; ++q) post[q] -= static_cast<int32_t>(o);
    }
    if (d) HIP_TRY(hipMemcpy(d, net->dly + so, mm, hipMemcpyDeviceToHost));
    if (wq) {
        if (net->params.wfmt == mc::kWFp32) {
            std::vector<float> f(static_cast<size_t>(mm));
            HIP_TRY(hipMemcpy(f.data(), static_cast<float *>(net->w) + so, mm * sizeof(float), hipMemcpyDeviceToHost));
            for (int64_t q = 0; q < mm; ++q) wq[q] = static_cast<int32_t>(std::nearbyint(static_cast<double>(f[q]) * 256.0));
        } else {
            std::vector<uint16_t> h(static_cast<size_t>(mm));
            HIP_TRY(hipMemcpy(h.data(), static_cast<uint16_t *>(net->w) + so, mm * sizeof(uint16_t), hipMemcpyDeviceToHost));
            for (int64_t q = 0; q < mm; ++q) {
                const double v = net->params.wfmt == mc::kWFp16 ? mc::half_value(h[q]) : mc::bf16_value(h[q]);
                wq[q] = static_cast<int32_t>(std::nearbyint(v * 256.0));
            }
        }
    }
    return MC_OK;
}

int mc_set_launch(mc_net *net, const mc_launch *l)
{
    if (!net || !l) return fail(MC_ERR_ARG, "net and l must not be NULL");
    LIVE_OR_FAIL(net);
    if (l->engine < 0 || l->engine > MC_ENGINE_TILED) return fail(MC_ERR_ARG, "unknown engine");
    if (l->tile && (l->tile < 16 || l->tile > 4096)) return fail(MC_ERR_ARG, "tile must be in [16, 4096]");
    if (l->ring < 0 || l->ring > 2) return fail(MC_ERR_ARG, "ring must be 0 (auto), 1 (LDS) or 2 (global)");
    if (l->graph_chunk && (l->graph_chunk < 1 || l->graph_chunk > 1024)) return fail(MC_ERR_ARG, "graph_chunk must be in [1, 1024]");
    if (l->seg && l->seg != 64 && l->seg != 128 && l->seg != 256 && l->seg != 512) return fail(MC_ERR_ARG, "seg must be 64, 128, 256 or 512");
    if (l->block && l->block != 64 && l->block != 128 && l->block != 256 && l->block != 512) return fail(MC_ERR_ARG, "block must be 64, 128, 256 or 512");
    if (l->deliver_grid < 0) return fail(MC_ERR_ARG, "deliver_grid must be >= 1");
    if (l->poll_delay < -1 || l->poll_delay > 255) return fail(MC_ERR_ARG, "poll_delay must be -1 or in [1, 255]");
    if (l->coop < 0 || l->coop > 2) return fail(MC_ERR_ARG, "coop must be 0 (keep), 1 (cooperative) or 2 (ordinary)");
    if (l->lanes < 0 || l->lanes > 64) return fail(MC_ERR_ARG, "lanes must be 0 (keep) or in [1, 64]");
    if (l->coop) net->coop = l->coop == 1;
    if (l->lanes) {
        net->lanes = l->lanes;
        net->lanes_set = true;
    }
    if (l->poll_delay) {
        net->poll_delay = l->poll_delay < 0 ? 0 : l->poll_delay;
        net->poll_delay_set = true;
    }
    bool changed = false;
    auto set = [&changed](int &dst, int v) { if (v && dst != v) { dst = v; changed = true; } };
    set(net->graph_chunk, l->graph_chunk);
    set(net->seg, l->seg);
    set(net->block, l->block);
    set(net->deliver_grid, l->deliver_grid);
    if (changed && net->graph_exec) {
        hipGraphExecDestroy(net->graph_exec);
        net->graph_exec = nullptr;
        net->graph_k = 0;
    }
    if (l->engine == MC_ENGINE_GRAPH) {
        net->engine = MC_ENGINE_GRAPH;
    } else if (l->engine == MC_ENGINE_TILED || ((l->tile || l->ring) && net->engine == MC_ENGINE_TILED) ||
               (l->engine == MC_ENGINE_AUTO && (l->tile || l->ring))) {
        int rc;
        if (!l->tile && !l->ring && !net->tile) {
            rc = setup_tiled_default(net);
        } else {
            // a new tile size without a ring choice picks the ring automatically;
            // a ring choice alone keeps the current tile size
            const int tile = l->tile ? l->tile : (net->tile ? net->tile : 256);
            const int ring = l->ring ? l->ring : (l->tile || !net->tile ? 0 : (net->tiled_shape.lds_ring ? 1 : 2));
            rc = setup_tiled(net, tile, ring);
        }
        if (rc) return rc;
        net->engine = MC_ENGINE_TILED;
    }
    return MC_OK;
}

int mc_set_step_budget(mc_net *net, double budget_us)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (!(budget_us >= 0.0) || budget_us > 2.0e7) return fail(MC_ERR_ARG, "budget_us must be in [0, 2e7]");
    const double ticks = std::nearbyint(budget_us * 100.0);        // s_memrealtime runs at 100 MHz
    net->budget_ticks = budget_us > 0.0 ? static_cast<uint32_t>(std::max(1.0, ticks)) : 0u;
    return MC_OK;
}

int mc_set_stream(mc_net *net, void *hip_stream)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    HIP_TRY(hipStreamSynchronize(net->stream));
    if (net->own_stream) HIP_TRY(hipStreamDestroy(net->stream));
    if (hip_stream) {
        net->stream = static_cast<hipStream_t>(hip_stream);
        net->own_stream = false;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking));
        net->own_stream = true;
    }
    return MC_OK;
}

int mc_set_trace(mc_net *net, int32_t steps)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (steps < 0 || steps > 65536) return fail(MC_ERR_ARG, "trace steps must be in [0, 65536]");
    if (net->trace) HIP_TRY(hipFree(net->trace));
    net->trace = nullptr;
    net->trace_steps = 0;
    net->trace_tiles = 0;
    if (steps == 0) return MC_OK;
    if (net->engine != MC_ENGINE_TILED) return fail(MC_ERR_UNSUPPORTED, "step tracing needs the TILED engine");
    // the step records plus one row of launch timestamps
    const size_t count = static_cast<size_t>(steps + 1) * net->n_tiles * mc::kTraceSlots;
    int rc = dalloc(&net->trace, count);
    if (rc) return rc;
    HIP_TRY(hipMemset(net->trace, 0, count * sizeof(uint64_t)));
    net->trace_steps = steps;
    net->trace_tiles = net->n_tiles;
    return MC_OK;
}

int mc_get_trace(mc_net *net, uint64_t *out, int64_t cap, int64_t *count)
{
    if (!net || !count) return fail(MC_ERR_ARG, "net and count must not be NULL");
    const int64_t n = static_cast<int64_t>(net->trace_steps + (net->trace_steps ? 1 : 0)) * net->trace_tiles * mc::kTraceSlots;
    *count = n;
    if (n == 0) return MC_OK;
    if (!out || cap < n) return fail(MC_ERR_BUFFER_TOO_SMALL, "buffer too small");
    HIP_TRY(hipMemcpy(out, net->trace, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
    return MC_OK;
}

int mc_inject_spikes(mc_net *net, int32_t instance, const int32_t *ids, int64_t count, int64_t *events_out)
{
    int64_t events = 0;
    int rc = inject_check(net, instance, ids, count, &events);
    if (rc) return rc;
    if (events_out) *events_out = events;
    if (count == 0) return MC_OK;
    if (count > net->inject_cap) {
        if (net->inject_buf) HIP_TRY(hipFree(net->inject_buf));
        net->inject_buf = nullptr;
        net->inject_cap = 0;
        if ((rc = dalloc(&net->inject_buf, count))) return rc;
        net->inject_cap = count;
    }
    return inject_run(net, instance, ids, count, net->inject_buf);
}

int mc_inject_spikes_noalloc(mc_net *net, int32_t instance, const int32_t *ids, int64_t count, int64_t *events_out)
{
    if (count > kNoAllocIds)
        return fail(MC_ERR_ARG, "count exceeds the " + std::to_string(kNoAllocIds) +
                                    " ids of the no-allocation staging array; use mc_inject_spikes");
    int64_t events = 0;
    const int rc = inject_check(net, instance, ids, count, &events);
    if (rc) return rc;
    if (!net->noalloc_ids) return fail(MC_ERR_HIP, "no-allocation staging array not resolved on this device");
    if (events_out) *events_out = events;
    if (count == 0) return MC_OK;
    return inject_run(net, instance, ids, count, net->noalloc_ids);
}

int mc_set_timing(mc_net *net, int32_t on)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (on && !net->timing) {
        LIVE_OR_FAIL(net);
        // The first elapsed-time query of an event pair costs the runtime some
        // tens of microseconds: pay it here for every pair a run may use, not
        // inside the first timed run.
        for (int b = 0; b < 3; ++b) {
            hipEvent_t e0 = b < 2 ? net->seg_ev0[b] : net->ev0, e1 = b < 2 ? net->seg_ev1[b] : net->ev1;
            float ms = 0.f;
            HIP_TRY(hipEventRecord(e0, net->stream));
            HIP_TRY(hipEventRecord(e1, net->stream));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        }
    }
    net->timing = on != 0;
    net->kernel_ms = 0.0;
    net->launches = 0;
    return MC_OK;
}

int mc_get_timing(mc_net *net, double *kernel_ms, int64_t *launches)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (kernel_ms) *kernel_ms = net->kernel_ms;
    if (launches) *launches = net->launches;
    return MC_OK;
}

int mc_tune(mc_net *net, int64_t trial_steps)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (trial_steps < 1 || trial_steps > 100000) return fail(MC_ERR_ARG, "trial_steps must be in [1, 100000]");
    LIVE_OR_FAIL(net);
    return autotune(net, trial_steps);
}

int mc_save_state(mc_net *net, const char *path)
{
    if (!net || !path) return fail(MC_ERR_ARG, "net and path must not be NULL");
    LIVE_OR_FAIL(net);
    return write_checkpoint(net, path);
}

int mc_load_state(mc_net *net, const char *path)
{
    if (!net || !path) return fail(MC_ERR_ARG, "net and path must not be NULL");
    return read_checkpoint(net, path);
}

int mc_probe(int32_t kind, int64_t bytes, double *rate, double *kernel_ms)
{
    if (!rate) return fail(MC_ERR_ARG, "rate must not be NULL");
    if (kind < MC_PROBE_HBM_COPY || kind > MC_PROBE_HBM_GATHER) return fail(MC_ERR_ARG, "unknown probe");
    if (kind != MC_PROBE_LDS_ATOMICS && (bytes < 8192 || bytes > (int64_t{1} << 36)))
        return fail(MC_ERR_ARG, "bytes must be in [8 KiB, 64 GiB]");
    double ms = 0.0;
    const hipError_t e = mc::run_probe(kind, bytes, rate, &ms);
    if (kernel_ms) *kernel_ms = ms;
    if (e == hipErrorOutOfMemory) return fail(MC_ERR_NOMEM, "probe buffer: out of device memory");
    if (e != hipSuccess) return fail(MC_ERR_HIP, std::string("probe: ") + hipGetErrorString(e));
    return MC_OK;
}

int mc_get_paths(mc_net *net, int64_t *counts, int32_t n)
{
    if (!net || !counts) return fail(MC_ERR_ARG, "net and counts must not be NULL");
    if (n < 1) return fail(MC_ERR_ARG, "n must be >= 1");
    unsigned long long c[mc::kPaths] = {};
    if (net->paths) {
        HIP_TRY(hipStreamSynchronize(net->stream));
        HIP_TRY(hipMemcpy(c, net->paths, sizeof(c), hipMemcpyDeviceToHost));
    }
    for (int32_t k = 0; k < n; ++k) counts[k] = k < mc::kPaths ? static_cast<int64_t>(c[k]) : 0;
    return MC_OK;
}

int mc_set_wait_limit(mc_net *net, int64_t polls)
{
    if (!net) return fail(MC_ERR_ARG, "net must not be NULL");
    if (polls < 0 || polls > int64_t{0xFFFFFFFF}) return fail(MC_ERR_ARG, "polls must be in [0, 2^32 - 1]");
    net->spin_limit = static_cast<uint32_t>(polls);
    return MC_OK;
}

void mc_free(mc_net *net) { release(net); }

}  // extern "C"
