// kernels.hip -- gfx950 kernels of one simulation step (global-memory form).
//
// Step n, per neuron i (Rhodes et al., arXiv 1909.08665):
//   * read and clear input-buffer slot n mod R (Sec. 3a(ii): the slot for the
//     current step is consumed and the buffer advances);
//   * add the step's Poisson background count times the background weight
//     (Sec. 3a(ii), source rates 8 Hz x K_ext, Sec. 3a(iii));
//   * exact integration of Eq. 1 (Sec. 2a): u <- P22 u + P21 I (+ P20 I_dc),
//     I <- P11 I + input, every product and sum rounded to float (no FMA);
//   * threshold test (u > theta), reset and refractory hold;
// then every spike's synaptic row is added into the targets' slots
// (n + delay) mod R with int32 atomics -- integer addition makes the result
// independent of the order in which rows are delivered.
//
// The input buffers are int32 in units of 1/256 pA; weights are stored as float
// (holding that fixed-point value), FP16 or BF16 and converted exactly.
#include <algorithm>

#include "kernels.hpp"
#include "philox_dev.hpp"

namespace mc {
namespace {

// Philox4x64-10 block for counter (c0, c1, 0, tag), key (seed, 0).
__device__ __forceinline__ void philox_block(uint64_t c0, uint64_t c1, uint64_t tag, uint64_t seed, uint64_t out[4])
{
    philox4x64(c0, c1, 0, tag, seed, out);
}

// 32-bit half h (0..7) of a block: high then low half of words 0, 1, 2, 3.
__device__ __forceinline__ uint32_t block_half(const uint64_t x[4], int h)
{
    const uint64_t w = h < 2 ? x[0] : h < 4 ? x[1] : h < 6 ? x[2] : x[3];
    return (h & 1) ? static_cast<uint32_t>(w) : static_cast<uint32_t>(w >> 32);
}

// Number of CDF thresholds not above a 32-bit uniform (inversion of the
// Poisson distribution).  The thresholds are non-decreasing, so this is the
// first k with v < thr[k]; the first eight are compared without branches
// (independent reads), the rest only when v passes the eighth.
__device__ __forceinline__ int poisson_count(uint32_t v, const uint64_t *thr)
{
    const uint64_t x = v;
    int k = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) k += x >= thr[j] ? 1 : 0;
    if (k == 8)
        while (k < kPoisMaxDev && x >= thr[k]) ++k;
    return k;
}

// Background spikes of neuron `local` at step n: one Philox block serves the
// eight neurons 8*(local/8) .. +7, each taking its own 32-bit half.
__device__ __forceinline__ int poisson_draw(uint64_t seed, int64_t n, int32_t local, const uint64_t *thr)
{
    uint64_t x[4];
    philox_block(static_cast<uint64_t>(n), static_cast<uint64_t>(local >> 3), 2, seed, x);
    return poisson_count(block_half(x, local & 7), thr);
}

template <int WF>
__device__ __forceinline__ int weight_q8(const void *__restrict__ w, uint64_t j)
{
    float f;
    if constexpr (WF == 0) {
        f = static_cast<const float *>(w)[j];
    } else if constexpr (WF == 1) {
        const uint16_t b = static_cast<const uint16_t *>(w)[j];
        f = static_cast<float>(__builtin_bit_cast(_Float16, b));
    } else {
        const uint16_t b = static_cast<const uint16_t *>(w)[j];
        f = __uint_as_float(static_cast<uint32_t>(b) << 16);
    }
    return __float2int_rn(f * 256.0f);   // exact: every stored weight is a multiple of 1/256 pA
}

// ---------------------------------------------------------------------------
// Neuron step: one lane per neuron; wavefront ballot compaction of spikes into
// the delivery work list (pre << 32 | chunk) and the spike recorder.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_neuron(DevNet P, int s_off)
{
    __shared__ uint64_t s_thr[8 * kPoisMaxDev];
    __shared__ unsigned long long s_pois[BLOCK / 64];
    for (int q = threadIdx.x; q < 8 * kPoisMaxDev; q += BLOCK) s_thr[q] = P.pois_thr[q];
    __syncthreads();

    StepCtl *ctl = P.ctl;
    const int64_t n = ctl->nbase + s_off;
    const int cur = static_cast<int>(n % 3);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->cnt[(n + 1) % 3] = 0;

    const int i = blockIdx.x * BLOCK + threadIdx.x;
    bool spike = false;
    int kpois = 0;
    uint32_t len = 0;
    if (i < P.n) {
        const uint32_t meta = P.meta[i];
        const int inst = static_cast<int>(meta >> 3), pop = static_cast<int>(meta & 7u);
        int32_t *cell = P.ring + static_cast<size_t>(n & P.ring_mask) * P.n + i;
        int32_t inq = *cell;
        *cell = 0;
        if (P.poisson_on) {
            kpois = poisson_draw(P.seeds[inst], n, i - P.inst_off[inst], s_thr + pop * kPoisMaxDev);
            inq += kpois * P.wq_ext;
        }
        const float in = __fmul_rn(__int2float_rn(inq), 0.00390625f);
        float u = P.u[i];
        float I = P.cur[i];
        int r = P.refr[i];
        if (r > 0) {
            r -= 1;
        } else {
            u = __fadd_rn(__fmul_rn(P.p22, u), __fmul_rn(P.p21, I));
            const float c = P.cdc[pop];
            if (c != 0.0f) u = __fadd_rn(u, c);
        }
        I = __fadd_rn(__fmul_rn(P.p11, I), in);
        if (u > P.theta) {
            spike = true;
            u = 0.0f;
            r = P.ref_steps;
            len = static_cast<uint32_t>(P.row_ptr[i + 1] - P.row_ptr[i]);
        }
        P.u[i] = u;
        P.cur[i] = I;
        P.refr[i] = static_cast<uint8_t>(r);
    }

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    // Background-event count of the block (no atomics: one slot per block).
    unsigned long long kp = static_cast<unsigned long long>(kpois);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kp += __shfl_xor(kp, o, 64);
    if (lane == 0) s_pois[wave] = kp;

    const unsigned long long mask = __ballot(spike);
    if (mask) {
        const uint32_t chunks = spike ? (len + static_cast<uint32_t>(P.seg) - 1) / static_cast<uint32_t>(P.seg) : 0;
        uint32_t incl = chunks;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const uint32_t wave_items = __shfl(incl, 63, 64);
        unsigned long long ev = len;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ev += __shfl_xor(ev, o, 64);
        const int leader = __ffsll(static_cast<long long>(mask)) - 1;
        const int nspk = __popcll(mask);
        unsigned long long old = 0;
        if (lane == leader) {
            old = atomicAdd(&ctl->cnt[cur], (static_cast<unsigned long long>(nspk) << 40) | wave_items);
            atomicAdd(&ctl->events, ev);
        }
        old = __shfl(old, leader, 64);
        if (spike) {
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            const int64_t pos = ctl->rec_total + static_cast<int64_t>(old >> 40) + rank;
            if (pos < P.rec_cap) {
                P.rec[pos] = rec_entry(n, i);
            } else {
                atomicOr(&ctl->flags, kFlagRecordOverflow);
            }
            const uint64_t first = (old & kMask40) + incl - chunks;
            for (uint32_t c = 0; c < chunks; ++c)
                P.work[first + c] = (static_cast<uint64_t>(i) << 32) | c;
        }
    }

    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (int q = 0; q < BLOCK / 64; ++q) s += s_pois[q];
        P.pois_acc[blockIdx.x] += s;
    }
}

// ---------------------------------------------------------------------------
// Delivery: one wavefront per work item (a chunk of `seg` consecutive synapses
// of one spiking row); coalesced loads of target / weight / delay, int32 atomic
// add into ring[(n + d) mod R][target].
// ---------------------------------------------------------------------------
template <int WF>
__global__ __launch_bounds__(256) void k_deliver(DevNet P, int s_off)
{
    StepCtl *ctl = P.ctl;
    const int64_t n = ctl->nbase + s_off;
    const unsigned long long c = ctl->cnt[n % 3];
    const uint64_t items = c & kMask40;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t S = static_cast<int32_t>(c >> 40);
        ctl->rec_total += S;
        if (S > ctl->max_s) ctl->max_s = S;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * 4;
    const int32_t *__restrict__ tgt = P.tgt;
    const uint8_t *__restrict__ dly = P.dly;
    int32_t *__restrict__ ring = P.ring;
    for (uint64_t it = static_cast<uint64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); it < items; it += nwaves) {
        const uint64_t wi = P.work[it];
        const int32_t pre = static_cast<int32_t>(wi >> 32);
        const uint64_t j0 = P.row_ptr[pre] + static_cast<uint64_t>(static_cast<uint32_t>(wi)) * static_cast<uint64_t>(P.seg);
        const uint64_t end = P.row_ptr[pre + 1];
        const uint64_t j1 = j0 + static_cast<uint64_t>(P.seg) < end ? j0 + static_cast<uint64_t>(P.seg) : end;
        for (uint64_t j = j0 + lane; j < j1; j += 64) {
            const int32_t t = tgt[j];
            const int32_t d = dly[j];
            const int wq = weight_q8<WF>(P.w, j);
            atomicAdd(ring + static_cast<size_t>((n + d) & P.ring_mask) * P.n + t, wq);
        }
    }
}

__global__ void k_advance(StepCtl *ctl, int steps)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->nbase += steps;
}

__global__ void k_clear_i32(int32_t *p, int64_t n)
{
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[q] = 0;
}

}  // namespace

hipError_t launch_neuron(const DevNet &d, int block, int s_off, hipStream_t st)
{
    const int grid = (d.n + block - 1) / block;
    switch (block) {
    case 64: hipLaunchKernelGGL(k_neuron<64>, dim3(grid), dim3(64), 0, st, d, s_off); break;
    case 128: hipLaunchKernelGGL(k_neuron<128>, dim3(grid), dim3(128), 0, st, d, s_off); break;
    case 256: hipLaunchKernelGGL(k_neuron<256>, dim3(grid), dim3(256), 0, st, d, s_off); break;
    case 512: hipLaunchKernelGGL(k_neuron<512>, dim3(grid), dim3(512), 0, st, d, s_off); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_deliver(const DevNet &d, int grid, int s_off, hipStream_t st)
{
    if (grid < 1) return hipErrorInvalidValue;
    switch (d.wfmt) {
    case 0: hipLaunchKernelGGL(k_deliver<0>, dim3(grid), dim3(256), 0, st, d, s_off); break;
    case 1: hipLaunchKernelGGL(k_deliver<1>, dim3(grid), dim3(256), 0, st, d, s_off); break;
    case 2: hipLaunchKernelGGL(k_deliver<2>, dim3(grid), dim3(256), 0, st, d, s_off); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_advance(const DevNet &d, int steps, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, d.ctl, steps);
    return hipGetLastError();
}

hipError_t launch_clear_i32(int32_t *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_clear_i32, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace mc

// ===========================================================================
// Tiled persistent engine.
//
// One workgroup per tile of consecutive neurons, all workgroups co-resident
// (cooperative launch); tiles never straddle two instances of a batch.  A
// workgroup keeps its tile's neuron state in registers and owns the tile's
// delay ring [R][len] -- in LDS when it fits, otherwise in global memory where
// no other workgroup ever touches it, so workgroup-scope atomics suffice.  The
// synapse rows stay in HBM; each spiking row is read once, every tile reading
// only the sub-row that targets its own neurons.  Per step:
//   1. update the tile (slot read/clear in LDS, Poisson, LIF), compact spikes;
//   2. publish the tile's spikes as self-tagged words (below);
//   3. draw the next step's Philox blocks (waves that do not poll) while the
//      other tiles publish;
//   4. wait until every tile's word of this step (tiles of the same instance)
//      is visible -- the step's only synchronisation -- and gather the ids;
//   5. read this tile's sub-row of every spiking row and add the weights into
//      the LDS ring with LDS integer atomics.
//
// Exchange protocol: each tile owns one 64-bit word per step parity,
//     bits 63..49 tag (n mod 32767) + 1, 48..36 spike count,
//     35..0 the offsets in the tile (12 bits each, tiles <= 4096) of its
//     first three spikes, first at bits 35..24,
// and, for its 4th, 5th, ... spikes, 64-bit entry words (tag32 = n + 1 | id);
// at full scale a tile almost never spikes more than three times in a step, so
// a step's ids arrive with the words and no entry has to be read.
// Words are written and polled with relaxed agent-scope atomics; a reader
// accepts a word only when its tag matches, so no fence or counter is needed:
// an aligned store is seen whole or not at all.  A tile cannot publish step
// n+2 (same parity) before it has seen every tile's step n+1 word, which every
// tile writes only after finishing its reads of step n, so within a launch the
// tag only has to tell step n from step n-2.  Between launches the words keep
// the tags of the last steps run; the host clears them only when the step
// index moved back (checkpoint load, tuner roll-back) or jumped so far ahead
// that an old tag could come round again, so a launch normally starts with no
// clearing at all.  The words of a step are polled by every tile of the
// instance; polling starts after a short sleep, since polls issued while the
// last tiles' stores are still in flight only congest the lines those stores
// go to.
// ===========================================================================
namespace mc {
namespace {

constexpr int kSpkBatch = 2048;              // spikes processed per delivery batch
constexpr int kSrcDirect = 16;               // most spikes of a tile mapped to their place one by one
constexpr int kGroupMin = 8;                 // fewest lanes per spike for delivery by fixed lane groups
constexpr int kWordIds = 3;                  // spike offsets carried by a tile's word
constexpr int kDeliverU = 4;                 // records in flight per thread in the step kernel's delivery
constexpr int kCursorU = 8;                  // and with a cursor over many spikes
constexpr int kRingBatch = 16;               // ring slots copied per round at launch start and end
constexpr int kInjectU = 4;                  // and in the injection kernel (16-byte chunks)
constexpr int kInjBatchMax = 8192;           // most spikes per batch of the injection kernel
constexpr int kInjWriteBack = 10;            // ring cells per thread in flight in the injection's write-back
constexpr size_t kLdsBytes = 160 * 1024;     // LDS of a compute unit (and the most one workgroup may use)
// LDS counted per workgroup in blocks of this size when bounding the
// workgroups a compute unit holds: larger than the allocation granularity, as
// a margin (three workgroups of 54.2 KB, 162.6 KB of the 160 KB, were not all
// placed; two of 65 KB and one of 102 KB are)
constexpr size_t kLdsBlock = 2048;

// Exclusive prefix sum of one value per thread, in thread order; returns the
// exclusive prefix and writes the block total to *total.  s_wave: >= 17 ints.
// Up to 8 waves, one barrier: every wave adds up the totals of the waves before
// it itself.  More waves: thread 0 turns the wave totals into offsets (two more
// barriers, fewer LDS reads).  The caller must pass a barrier before the next
// call reuses s_wave.
__device__ __forceinline__ int block_scan_excl(int v, int *s_wave, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int x = __shfl_up(incl, o, 64);
        if (lane >= o) incl += x;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    if (nwaves <= 8) {
        int before = 0, all = 0;
        for (int q = 0; q < nwaves; ++q) {
            const int x = s_wave[q];
            before += q < wave ? x : 0;
            all += x;
        }
        *total = all;
        return before + incl - v;
    }
    if (threadIdx.x == 0) {
        int run = 0;
        for (int q = 0; q < nwaves; ++q) {
            const int x = s_wave[q];
            s_wave[q] = run;
            run += x;
        }
        s_wave[16] = run;
    }
    __syncthreads();
    *total = s_wave[16];
    return s_wave[wave] + incl - v;
}

// In-place exclusive scan of a[0..count) in LDS; a[count] receives the total.
__device__ void lds_scan_excl(int *a, int count, int *s_wave)
{
    const int per = (count + blockDim.x - 1) / blockDim.x;
    const int beg = min(count, static_cast<int>(threadIdx.x) * per);
    const int end = min(count, beg + per);
    int sum = 0;
    for (int q = beg; q < end; ++q) sum += a[q];
    int total;
    int run = block_scan_excl(sum, s_wave, &total);
    for (int q = beg; q < end; ++q) {
        const int x = a[q];
        a[q] = run;
        run += x;
    }
    if (threadIdx.x == 0) a[count] = total;
    __syncthreads();
}

// Largest q in [0, n) with a[q] <= key (a nondecreasing, a[0] <= key).
__device__ __forceinline__ int find_segment(const int *a, int n, int key)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

template <class W>
__device__ __forceinline__ W load_word(const W *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class W>
__device__ __forceinline__ void store_word(W *p, W v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile word of step n: bits 63..49 a tag from the step index ((n mod 32767) + 1,
// never 0), 48..36 the tile's spike count, then the 12-bit offsets in the tile
// of its first three spikes from bit 35 down.
__device__ __forceinline__ uint64_t word_tag(int64_t n) { return static_cast<uint64_t>(n % 32767) + 1u; }
__device__ __forceinline__ bool word_is(uint64_t w, uint64_t tag) { return (w >> 49) == tag; }
__device__ __forceinline__ int word_count(uint64_t w) { return static_cast<int>((w >> 36) & 0x1FFFu); }
__device__ __forceinline__ int word_offset(uint64_t w, int k) { return static_cast<int>((w >> (24 - 12 * k)) & 0xFFFu); }
__device__ __forceinline__ uint64_t word_make(uint64_t tag, int count) { return (tag << 49) | (static_cast<uint64_t>(count) << 36); }

// Give up the launch: name it in the abort word (the other workgroups' waits
// see it and give up too) and flag the time-out for the host.
__device__ __forceinline__ void give_up(const TiledNet &P)
{
    __hip_atomic_store(P.abort_word, P.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicOr(&P.head->flags, kFlagTimeout);
}

// Poll *p until `accept(word)`; false if the wait was abandoned: after
// spin_limit polls (checked every 1024; a limit of 0 gives up at once, which
// lets the host test the failure path), or when another workgroup of this
// launch gave up.
template <class W, class Accept>
__device__ __forceinline__ bool wait_word(const W *p, const TiledNet &P, Accept accept, W &w)
{
    if (P.spin_limit == 0) {
        give_up(P);
        return false;
    }
    uint32_t spins = 0;
    for (;;) {
        w = load_word(p);
        if (accept(w)) return true;
        if ((++spins & 1023u) == 0) {
            if (__hip_atomic_load(P.abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == P.epoch)
                return false;
            if (spins > P.spin_limit) {
                give_up(P);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Decode packed synapse record j: tile-local target, delay, weight in 1/256 pA.
template <int SF>
__device__ __forceinline__ int syn_record(const void *__restrict__ syn, uint32_t j, int &local, int &d)
{
    float f;
    if constexpr (SF <= kSyn8BF16) {
        const uint2 r = static_cast<const uint2 *>(syn)[j];
        local = static_cast<int>(r.x & 0xFFFFu);
        d = static_cast<int>((r.x >> 16) & 0xFFu);
        if constexpr (SF == kSyn8F32) f = __uint_as_float(r.y);
        else if constexpr (SF == kSyn8F16) f = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(r.y)));
        else f = __uint_as_float(r.y << 16);
    } else {
        const uint32_t r = static_cast<const uint32_t *>(syn)[j];
        local = static_cast<int>(r & 0x3FFu);
        d = static_cast<int>((r >> 10) & 0x3Fu);
        if constexpr (SF == kSyn4F16) f = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(r >> 16)));
        else f = __uint_as_float(r & 0xFFFF0000u);
    }
    return __float2int_rn(f * 256.0f);
}

// Decode a record from its raw bits (8 or 4 bytes, widened), loaded apart
// from its decoding so that the load can be issued well before.
template <int SF>
__device__ __forceinline__ int rec_decode(uint64_t raw, int &local, int &d)
{
    float f;
    if constexpr (SF <= kSyn8BF16) {
        const uint32_t x = static_cast<uint32_t>(raw), y = static_cast<uint32_t>(raw >> 32);
        local = static_cast<int>(x & 0xFFFFu);
        d = static_cast<int>((x >> 16) & 0xFFu);
        if constexpr (SF == kSyn8F32) f = __uint_as_float(y);
        else if constexpr (SF == kSyn8F16) f = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(y)));
        else f = __uint_as_float(y << 16);
    } else {
        const uint32_t r = static_cast<uint32_t>(raw);
        local = static_cast<int>(r & 0x3FFu);
        d = static_cast<int>((r >> 10) & 0x3Fu);
        if constexpr (SF == kSyn4F16) f = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(r >> 16)));
        else f = __uint_as_float(r & 0xFFFF0000u);
    }
    return __float2int_rn(f * 256.0f);
}

// Add the events of nb spikes into a ring: spike q's sub-row is records
// s_beg[q] .. s_beg[q] + len - 1, s_pre the exclusive prefix of the lengths
// (s_pre[nb] = E), so event e belongs to the last q with s_pre[q] <= e.
// Thread l takes events l, l + nthr, ... in rounds of U (consecutive lanes read
// consecutive records): it finds their spikes (independent binary searches in
// LDS), loads all U records, then adds them -- U loads in flight per thread
// and no barrier, whatever the mix of sub-row lengths.  add(target, delay, wq)
// does the ring update.  With a budget (100 MHz ticks since t_step, 0 for
// none), a wave that finds the budget spent before a round stops and adds the
// number of its threads' remaining events to `dropped`.
template <int SF, int U, class Add>
__device__ __forceinline__ void deliver_events(const void *__restrict__ syn, const int *s_beg, const int *s_pre, int nb,
                                               int E, Add add, uint64_t t_step = 0, uint32_t budget = 0,
                                               unsigned long long *dropped = nullptr)
{
    const int l = threadIdx.x, nthr = blockDim.x;
    for (int e0 = 0; e0 < E; e0 += U * nthr) {
        if (budget && __builtin_amdgcn_s_memrealtime() - t_step > budget) {
            if (e0 + l < E) *dropped += static_cast<unsigned long long>((E - (e0 + l) + nthr - 1) / nthr);
            return;
        }
        uint32_t j[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int e = e0 + l + k * nthr;
            const int q = e < E ? find_segment(s_pre, nb + 1, e) : 0;
            j[k] = e < E ? static_cast<uint32_t>(s_beg[q]) + static_cast<uint32_t>(e - s_pre[q]) : 0u;
        }
        int wq[U], tg[U], d[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (e0 + l + k * nthr < E) wq[k] = syn_record<SF>(syn, j[k], tg[k], d[k]);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (e0 + l + k * nthr < E) add(tg[k], d[k], wq[k]);
    }
}

// Add the events of nb spikes, spike q's sub-row being records s_beg[q] ..
// s_beg[q] + s_len[q] - 1, with a fixed group of nthr / nb lanes per spike:
// lane r of spike q's group takes records r, r + group, ... (U in flight), so
// no scan of the lengths and no search for an event's spike.  Balanced when
// the sub-rows are about equally long and the groups are wide (the caller
// ensures nb * 8 <= nthr).  Returns the records this thread added.
template <int SF, int U, class Add>
__device__ __forceinline__ unsigned long long deliver_grouped(const void *__restrict__ syn, const int *s_beg,
                                                              const int *s_len, int nb, Add add)
{
    const int l = threadIdx.x, group = static_cast<int>(blockDim.x) / nb;
    const int q = l / group, r = l - q * group;
    if (q >= nb) return 0;
    const uint32_t beg = static_cast<uint32_t>(s_beg[q]);
    const int len = s_len[q];
    for (int j0 = r; j0 < len; j0 += U * group) {
        int wq[U], tg[U], d[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (j0 + k * group < len) wq[k] = syn_record<SF>(syn, beg + static_cast<uint32_t>(j0 + k * group), tg[k], d[k]);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (j0 + k * group < len) add(tg[k], d[k], wq[k]);
    }
    return r < len ? static_cast<unsigned long long>((len - r + group - 1) / group) : 0ull;
}

// Add the events of nb spikes, spike q's sub-row being records s_beg[q] ..
// s_beg[q] + s_len[q] - 1, with groups of G lanes: group g (of nthr / G) takes
// spikes g, g + groups, ..., each in chunks of G consecutive records, lane r
// of the group taking record r of the chunk.  The group's cursor (spike,
// chunk) is the same in all its lanes, so each load instruction reads G
// consecutive records per group (one or two cache lines), and each lane keeps
// U records in flight; there is neither a scan of the lengths nor a search
// for an event's spike.  Lanes past a sub-row's end idle for that chunk.
// Returns the records this thread added.
template <int SF, int U, class Add>
__device__ __forceinline__ unsigned long long deliver_cursor(const void *__restrict__ syn, const int *s_beg,
                                                             const int *s_len, int nb, int G, Add add)
{
    const int l = threadIdx.x, groups = static_cast<int>(blockDim.x) / G;
    int q = l / G;
    const int r = l - q * G;
    if (q >= groups) return 0;                         // lanes past the last whole group
    int j0 = 0, len = 0;
    uint32_t beg = 0;                                  // record indices are unsigned 32-bit
    auto next_row = [&](int from) {                    // the group's next spike with records, from `from` on
        for (q = from; q < nb; q += groups) {
            len = s_len[q];
            if (len > 0) {
                beg = static_cast<uint32_t>(s_beg[q]);
                return;
            }
        }
    };
    next_row(q);
    unsigned long long done = 0;
    while (q < nb) {
        uint32_t idx[U];
        bool v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            v[k] = q < nb && j0 + r < len;
            idx[k] = v[k] ? beg + static_cast<uint32_t>(j0 + r) : 0u;
            if (q < nb) {
                j0 += G;
                if (j0 >= len) {
                    j0 = 0;
                    next_row(q + groups);
                }
            }
        }
        int wq[U], tg[U], d[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (v[k]) wq[k] = syn_record<SF>(syn, idx[k], tg[k], d[k]);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (v[k]) {
                add(tg[k], d[k], wq[k]);
                ++done;
            }
    }
    return done;
}

// The lane-group cursor of deliver_cursor for long spike lists, reading the
// store in aligned 16-byte chunks (two 8-byte or four 4-byte records): lane r
// of a group takes chunk j0 + r of the spike's sub-row, so that a group's load
// covers G x 16 consecutive bytes, and a round of U chunks per lane needs half
// (or a quarter) of the loads and cursor steps of one record per load.  A chunk
// at either end of a sub-row also holds records of the neighbouring sub-rows: a
// per-chunk mask keeps only the spike's own.  Two sets of U chunks: the loads
// of the next round are issued before the current round is decoded and added,
// so the memory system always has a round in flight.  The store must be
// allocated to a whole number of 16-byte chunks.  s_row[q] = (first record,
// length) of spike q's sub-row, read as one word.  Returns the records this
// thread added.
template <int SF, int U, class Add>
__device__ __forceinline__ unsigned long long deliver_chunks_pipelined(const void *__restrict__ syn, const int2 *s_row,
                                                                       int nb, int G, Add add)
{
    constexpr int P = SF <= kSyn8BF16 ? 2 : 4;         // records per chunk
    const int l = threadIdx.x, groups = static_cast<int>(blockDim.x) / G;
    int q = l / G;
    const int r = l - q * G;
    if (q >= groups) return 0;
    // sub-row [lo, hi): chunks c0 .. c0 + nch - 1 (record indices are unsigned
    // 32-bit: a store may hold up to 2^32 - 1 records)
    int j0 = 0, nch = 0;
    uint32_t lo = 0, hi = 0, c0 = 0;
    auto next_row = [&](int from) {
        for (q = from; q < nb; q += groups) {
            const int2 row = s_row[q];
            if (row.y > 0) {
                lo = static_cast<uint32_t>(row.x);
                hi = lo + static_cast<uint32_t>(row.y);
                c0 = lo / P;
                nch = static_cast<int>((hi - 1) / P + 1 - c0);
                return;
            }
        }
    };
    const uint4 *chunks = static_cast<const uint4 *>(syn);
    // the cursor's next U chunks: their loads, and the mask of the records of
    // each that belong to its spike (0 for an idle lane, which reads chunk 0)
    auto fill = [&](uint4 (&raw)[U], int (&m)[U]) {
        uint32_t idx[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            m[k] = 0;
            idx[k] = 0u;
            if (q < nb) {
                if (j0 + r < nch) {
                    const uint32_t c = c0 + static_cast<uint32_t>(j0 + r), base = c * P;   // base <= hi - 1
                    const int first = lo > base ? static_cast<int>(lo - base) : 0;
                    const int last = hi - base < static_cast<uint32_t>(P) ? static_cast<int>(hi - base) : P;
                    m[k] = ((1 << last) - 1) & ~((1 << first) - 1);
                    idx[k] = c;
                }
                j0 += G;
                if (j0 >= nch) {
                    j0 = 0;
                    next_row(q + groups);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) raw[k] = chunks[idx[k]];
    };
    unsigned long long done = 0;
    auto one = [&](uint64_t rec) {
        int tg, d;
        const int wq = rec_decode<SF>(rec, tg, d);
        add(tg, d, wq);
        ++done;
    };
    auto consume = [&](const uint4 (&raw)[U], const int (&m)[U]) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if constexpr (P == 2) {
                if (m[k] & 1) one((static_cast<uint64_t>(raw[k].y) << 32) | raw[k].x);
                if (m[k] & 2) one((static_cast<uint64_t>(raw[k].w) << 32) | raw[k].z);
            } else {
                if (m[k] & 1) one(raw[k].x);
                if (m[k] & 2) one(raw[k].y);
                if (m[k] & 4) one(raw[k].z);
                if (m[k] & 8) one(raw[k].w);
            }
        }
    };
    next_row(q);
    uint4 ra[U], rb[U];
    int ma[U], mb[U];
    fill(ra, ma);
    for (;;) {
        bool more = q < nb;
        fill(rb, mb);
        consume(ra, ma);
        if (!more) break;
        more = q < nb;
        fill(ra, ma);
        consume(rb, mb);
        if (!more) break;
    }
    return done;
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD b mod 8),
// each XCD with its own L2.  Workgroup b takes tile rank(b) in the order
// (b mod 8, b / 8), so that every XCD holds a contiguous run of tiles: the
// cache lines that neighbouring tiles' sub-rows and sub-row entries share are
// then fetched into one L2.  A bijection of [0, n); speed only.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int x = b % kXcds;
    int base = 0;
    for (int y = 0; y < x; ++y) base += (n - y + kXcds - 1) / kXcds;
    return base + b / kXcds;
}

// MODE bit 0: the lossy real-time form (P.budget_ticks > 0); bit 1: the
// per-step phase trace (P.trace set).  Separate instantiations, so that the
// plain step kernel carries none of their state (each costs it ~3 % in scalar
// register pressure).
template <int SF, bool LRING, int NPT, int MODE>
__global__ __launch_bounds__(1024) void k_tiled(TiledNet P, int64_t steps)
{
    constexpr bool BUDGET = (MODE & 1) != 0, TRACE = (MODE & 2) != 0;
    extern __shared__ int lds[];
    __shared__ uint64_t s_thr[8 * kPoisMaxDev];
    __shared__ int s_wave[17];
    __shared__ int s_wave2[17];                        // the wait's scan: waves may still read s_wave
    __shared__ uint64_t s_mask[16];                    // spike mask of each wave (one neuron per thread)
    __shared__ int s_abort;
    __shared__ int s_big;                              // step in which some tile sent over kSrcDirect spikes
    __shared__ int s_many;                             // step in which some tile sent over kWordIds spikes
    __shared__ long long s_recbase;
    __shared__ unsigned long long s_drop;              // events dropped by the step budget (this launch)
    __shared__ uint32_t s_paths[kPaths];               // tile-steps per delivery path (this launch)

    const DevNet &B = P.base;
    StepCtl *ctl = B.ctl;
    const int t = xcd_tile(blockIdx.x, gridDim.x), tmax = P.tile_max;
    const TileDesc td = P.tiles[t];
    const int tl = t - td.itile0, T = td.intiles;     // local tile index, tiles of the instance
    const int l = threadIdx.x, nthr = blockDim.x;
    const int mask = B.ring_mask, R = mask + 1;
    const int32_t t0 = td.t0;
    const int tlen = td.len;

    // Global-ring variant: the ring lives in this workgroup's private, cache-line
    // aligned slice of global memory, and the nearest W slots also have an LDS
    // row each: an event whose delay is at most W is added there, and the update
    // sums both parts of its slot.  At step n (after its update) the window rows
    // hold slots n + 1 .. n + W, slot s in row s mod W.
    const int W = LRING ? 0 : P.win;
    int *ring = lds;                                   // [R][tmax] when LRING, else the [W][tmax] window
    int32_t *gring = LRING ? nullptr : P.gring + static_cast<size_t>(t) * R * P.gstride;
    // [2][tmax/8 + 2][4] Philox blocks of steps n + 1 and n + 2 (by step parity),
    // one per group of 8 neurons (8-byte aligned: the ring part is rounded to even)
    const int nbk = tmax / 8 + 2;
    uint64_t *s_blk = reinterpret_cast<uint64_t *>(lds + (LRING ? R * tmax : ((W * tmax + 1) & ~1)));
    uint64_t *s_word = s_blk + 2 * 4 * nbk;            // [T] this step's word of every tile of the instance
    int *s_cnt = reinterpret_cast<int *>(s_word + P.max_intiles);   // [T + 1] spike counts -> offsets
    int *s_beg = s_cnt + P.max_intiles + 1;            // [kSpkBatch] sub-row start
    int *s_pre = s_beg + kSpkBatch;                    // [kSpkBatch + 1] sub-row lengths -> offsets
    int *s_own = s_pre + kSpkBatch + 1;                // [tmax] this tile's spikes
    // Between the wait and the ids phase s_beg[g] holds (tile << 16 | index in
    // it) of spike g of the first batch; each thread reads the entries it then
    // overwrites with sub-row starts.
    int *s_src = s_beg;

    for (int q = l; q < 8 * kPoisMaxDev; q += nthr) s_thr[q] = B.pois_thr[q];
    // trace form: launch timestamps of this tile (entry, first step, after the
    // last step, exit) in the row after the step records
    uint64_t *tr_launch = TRACE && l == 0 && P.trace ? P.trace + (static_cast<size_t>(P.trace_steps) * P.n_tiles + t) * kTraceSlots
                                                      : nullptr;
    if (tr_launch) tr_launch[0] = __builtin_amdgcn_s_memrealtime();
    // The tile's part of the ring, kRingBatch slots' loads in flight at a time
    // (one dependent round trip per slot would cost the launch tens of us).
    for (int s0 = 0; s0 < R; s0 += kRingBatch)
        for (int q = l; q < (LRING ? tmax : tlen); q += nthr) {
            int v[kRingBatch];
#pragma unroll
            for (int k = 0; k < kRingBatch; ++k)
                v[k] = s0 + k < R && q < tlen ? B.ring[static_cast<size_t>(s0 + k) * B.n + t0 + q] : 0;
#pragma unroll
            for (int k = 0; k < kRingBatch; ++k)
                if (s0 + k < R) {
                    if (LRING) ring[(s0 + k) * tmax + q] = v[k];
                    else gring[(s0 + k) * P.gstride + q] = v[k];
                }
        }
    for (int q = l; q < W * tmax; q += nthr) ring[q] = 0;
    if (l == 0) {
        s_abort = 0;
        s_big = -1;
        s_many = -1;
        s_drop = 0;
        for (int k = 0; k < kPaths; ++k) s_paths[k] = 0;
    }

    // The tile lies in one instance: its seed and local numbering are uniform.
    const uint64_t seed = B.seeds[B.meta[t0] >> 3];
    const int32_t lo_local = t0 - td.inst_n0;
    // Background input is pipelined over two steps: while step n waits for the
    // other tiles, the highest threads draw the Philox blocks of step n + 2 (one
    // per group of 8 neurons; at full scale in a wave that does not poll), and
    // every thread turns the blocks of step n + 1, drawn a step earlier, into
    // its neurons' counts.
    const int g0 = lo_local >> 3, ng = ((lo_local + tlen - 1) >> 3) - g0 + 1;
    auto fill_blocks = [&](int64_t m) {
        uint64_t *dst = s_blk + static_cast<size_t>(m & 1) * 4 * nbk;
        for (int j = nthr - 1 - l; j < ng; j += nthr) {
            uint64_t x[4];
            philox_block(static_cast<uint64_t>(m), static_cast<uint64_t>(g0 + j), 2, seed, x);
#pragma unroll
            for (int w = 0; w < 4; ++w) dst[4 * j + w] = x[w];
        }
    };

    // neurons l, l + nthr, ... of the tile
    float u[NPT], I[NPT], cdc[NPT];
    int r[NPT], pop[NPT], kp[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = l + k * nthr;
        u[k] = I[k] = cdc[k] = 0.f;
        r[k] = pop[k] = kp[k] = 0;
        if (q < tlen) {
            const int32_t i = t0 + q;
            u[k] = B.u[i];
            I[k] = B.cur[i];
            r[k] = B.refr[i];
            pop[k] = static_cast<int>(B.meta[i] & 7u);
            cdc[k] = B.cdc[pop[k]];
        }
    }
    int64_t n = ctl->nbase;
    int64_t rec_base = 0;                              // this launch's recorder starts empty
    unsigned long long ev_acc = 0, pois_sum = 0, drop_acc = 0;
    auto counts = [&](int64_t m) {
        const uint64_t *src = s_blk + static_cast<size_t>(m & 1) * 4 * nbk;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int loc = lo_local + l + k * nthr;
            if (l + k * nthr < tlen) {
                const uint64_t wd = src[4 * ((loc >> 3) - g0) + ((loc & 7) >> 1)];
                kp[k] = poisson_count((loc & 1) ? static_cast<uint32_t>(wd) : static_cast<uint32_t>(wd >> 32),
                                      s_thr + pop[k] * kPoisMaxDev);
            }
        }
    };
    __syncthreads();
    if (B.poisson_on) {
        fill_blocks(n);
        fill_blocks(n + 1);
    }
    __syncthreads();
    if (B.poisson_on) counts(n);

    // Optional per-step phase timestamps (100 MHz constant clock), thread 0 only:
    // 0 step start, 1 spikes published, 2 Philox block of step n + 2 and counts
    // of step n + 1 done (by the last thread, which draws the tile's first
    // block), 3 wait begins,
    // 4 every tile's word seen, 5 spike ids gathered, 6 delivery done,
    // 7 spike count of the step (this tile's instance).
    uint64_t *tr = nullptr;
    if (tr_launch) tr_launch[1] = __builtin_amdgcn_s_memrealtime();
    for (int64_t s = 0; s < steps; ++s, ++n) {
        const int par = static_cast<int>(n & 1);
        const uint64_t tag15 = word_tag(n);
        const uint64_t tag32 = static_cast<uint64_t>(static_cast<uint32_t>(n + 1));
        uint64_t *words = P.xchg + static_cast<size_t>(par) * P.n_tiles + td.itile0;
        uint64_t *entries = P.xent + (static_cast<size_t>(par) * P.n_tiles + td.itile0) * tmax;
        const int slot = static_cast<int>(n & mask);
        const int wslot = W ? static_cast<int>(n % W) : 0;
        const uint64_t t_step = BUDGET ? __builtin_amdgcn_s_memrealtime() : 0;
        tr = (TRACE && l == 0 && s < P.trace_steps) ? P.trace + (static_cast<size_t>(s) * P.n_tiles + t) * kTraceSlots
                                                      : nullptr;
        uint64_t *tr_blk = (TRACE && l == nthr - 1 && s < P.trace_steps)
                               ? P.trace + (static_cast<size_t>(s) * P.n_tiles + t) * kTraceSlots : nullptr;
        if (tr) tr[0] = __builtin_amdgcn_s_memrealtime();
        // ---- 1. neuron update ------------------------------------------------
        bool spike[NPT];
        int nmine = 0;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int q = l + k * nthr;
            spike[k] = false;
            if (q < tlen) {
                int inq;
                if (LRING) {
                    int *cell = ring + slot * tmax + q;
                    inq = *cell;
                    *cell = 0;
                } else {
                    int32_t *cell = gring + slot * P.gstride + q;
                    inq = *cell;
                    *cell = 0;
                    if (W) {
                        int *wc = ring + wslot * tmax + q;
                        inq += *wc;
                        *wc = 0;
                    }
                }
                inq += kp[k] * B.wq_ext;
                pois_sum += static_cast<unsigned long long>(kp[k]);
                const float in = __fmul_rn(__int2float_rn(inq), 0.00390625f);
                if (r[k] > 0) {
                    r[k] -= 1;
                } else {
                    u[k] = __fadd_rn(__fmul_rn(B.p22, u[k]), __fmul_rn(B.p21, I[k]));
                    if (cdc[k] != 0.0f) u[k] = __fadd_rn(u[k], cdc[k]);
                }
                I[k] = __fadd_rn(__fmul_rn(B.p11, I[k]), in);
                if (u[k] > B.theta) {
                    spike[k] = true;
                    u[k] = 0.0f;
                    r[k] = B.ref_steps;
                    ++nmine;
                }
            }
        }
        // ---- 2. compaction and publication ---------------------------------------
        // One neuron per thread: each wave leaves its spike mask beside its count,
        // so thread 0 finds the first spikes right after the scan's barrier and
        // publishes the word without waiting for the compacted list.
        if (NPT == 1) {
            const uint64_t m = __ballot(spike[0]);
            if ((l & 63) == 0) s_mask[l >> 6] = m;
        }
        int nspk;
        int pos = block_scan_excl(nmine, s_wave, &nspk);
        if (NPT == 1 && l == 0) {
            uint64_t w = word_make(tag15, nspk);
            const int nw = min(nspk, kWordIds);
            for (int q = 0, got = 0; got < nw; ++q) {
                for (uint64_t m = s_mask[q]; m && got < nw; m &= m - 1, ++got)
                    w |= static_cast<uint64_t>(q * 64 + __builtin_ctzll(m)) << (24 - 12 * got);
            }
            store_word(words + tl, w);
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (spike[k]) {
                const int32_t i = t0 + l + k * nthr;
                s_own[pos] = i;
                if (pos >= kWordIds)
                    store_word(entries + static_cast<size_t>(tl) * tmax + pos, (tag32 << 32) | static_cast<uint32_t>(i));
                ++pos;
            }
        }
        if (NPT != 1) {
            __syncthreads();
            if (l == 0) {
                uint64_t w = word_make(tag15, nspk);
                for (int k = 0; k < min(nspk, kWordIds); ++k)
                    w |= static_cast<uint64_t>(s_own[k] - t0) << (24 - 12 * k);
                store_word(words + tl, w);
            }
        }
        if (tr) tr[1] = __builtin_amdgcn_s_memrealtime();
        // Batch, several neurons per thread: reserve this step's range of the
        // recorder now, from the last thread (which polls only when every thread
        // does), so that the atomic's round trip overlaps the wait; its result
        // goes to LDS before the wait's barrier.  (The one-neuron-per-thread
        // form reserves after the wait: the early form costs it 3 %.)
        const bool rec_reserve = NPT > 1 && T != P.n_tiles && nspk > 0 && l == nthr - 1;
        unsigned long long rec_reserved = 0;
        if (rec_reserve)
            rec_reserved = atomicAdd(&P.head->rec_total, static_cast<unsigned long long>(nspk));
        // ---- 3. background input: blocks of step n + 2 into the buffer whose
        // blocks (step n) were all turned into counts before the last barrier;
        // counts of step n + 1 from blocks drawn in the previous step -----------
        if (tr) tr[3] = __builtin_amdgcn_s_memrealtime();
        if (B.poisson_on) {
            fill_blocks(n + 2);
            counts(n + 1);
        }
        if (tr_blk) tr_blk[2] = __builtin_amdgcn_s_memrealtime();
        // ---- 4. every tile's word of this step: counts and first ids --------------
        if (rec_reserve) s_recbase = static_cast<long long>(rec_reserved);
        // this tile's spikes into its range of the recorder (batch)
        auto record_reserved = [&]() {
            for (int q = l; q < nspk; q += nthr) {
                const int64_t at = s_recbase + q;
                if (at < B.rec_cap) B.rec[at] = rec_entry(n, s_own[q]);
                else atomicOr(&P.head->flags, kFlagRecordOverflow);
            }
        };
        // a range reserved before the wait is filled even when the wait is
        // abandoned, so that the recorder never holds unwritten entries
        const bool reserved_early = NPT > 1 && T != P.n_tiles && nspk > 0;
        if (l < T)
            for (int z = 0; z < P.poll_delay; ++z) __builtin_amdgcn_s_sleep(1);
        // One neuron per thread: the poller of tile l loads the sub-rows of l's
        // first spikes (ids in l's word) as soon as its wave has every word, and
        // the loads stay in flight through the count scan and its barriers.
        uint2 sr_first[kWordIds];
        int nk = 0, ex_l = 0;
        if (T <= nthr) {
            // one word per thread: scan the counts straight from the registers
            int c = 0;
            if (l < T) {
                uint64_t w = 0;
                if (wait_word(words + l, P, [tag15](uint64_t x) { return word_is(x, tag15); }, w)) {
                    c = word_count(w);
                    s_word[l] = w;
                    if (NPT == 1) {
                        nk = min(c, kWordIds);
                        const int64_t sub_l = td.sub_base + static_cast<int64_t>(l) * td.stride * T;
#pragma unroll
                        for (int k = 0; k < kWordIds; ++k)
                            if (k < nk) sr_first[k] = P.subrow[sub_l + static_cast<int64_t>(word_offset(w, k)) * T];
                    }
                } else {
                    s_abort = 1;
                }
            }
            int total;
            const int ex = block_scan_excl(c, s_wave2, &total);
            ex_l = ex;
            if (NPT == 1 && c > kWordIds) s_many = static_cast<int>(n);
            if (l < T) {
                s_cnt[l] = ex;
                // spike ex + k of the step is spike k of tile l (the first batch; a
                // tile with more spikes sends the step to the binary search instead).
                // Tiles of one neuron per thread only: the instance has many tiles.
                if (NPT > 1) {
                } else if (c <= kSrcDirect) {
                    for (int k = 0; k < c && ex + k < kSpkBatch; ++k) s_src[ex + k] = (l << 16) | k;
                } else {
                    s_big = static_cast<int>(n);
                }
            }
            if (l == 0) s_cnt[T] = total;
            __syncthreads();
            if (s_abort) {
                if (reserved_early) record_reserved();
                break;
            }
        } else {
            for (int q = l; q < T; q += nthr) {
                uint64_t w = 0;
                if (!wait_word(words + q, P, [tag15](uint64_t x) { return word_is(x, tag15); }, w)) {
                    s_abort = 1;
                    break;
                }
                s_cnt[q] = word_count(w);
                s_word[q] = w;
            }
            __syncthreads();
            if (s_abort) {
                if (reserved_early) record_reserved();
                break;
            }
            lds_scan_excl(s_cnt, T, s_wave2);
        }
        const int S = s_cnt[T];
        if (tr) {
            tr[4] = __builtin_amdgcn_s_memrealtime();
            tr[7] = static_cast<uint64_t>(S);
        }
        // record this tile's spikes.  One instance: every tile knows every count,
        // so its place in the step's list is fixed without atomics.  Batch: each
        // spiking tile reserves its range with one atomic.
        if (T == P.n_tiles) {
            for (int q = l; q < nspk; q += nthr) {
                const int64_t at = rec_base + s_cnt[tl] + q;
                if (at < B.rec_cap) B.rec[at] = rec_entry(n, s_own[q]);
                else atomicOr(&P.head->flags, kFlagRecordOverflow);
            }
            rec_base += S;
        } else if (nspk) {
            if (NPT == 1) {
                if (l == 0)
                    s_recbase = static_cast<long long>(atomicAdd(&P.head->rec_total,
                                                                 static_cast<unsigned long long>(nspk)));
                __syncthreads();
            }   // else reserved before the wait (s_recbase written before its barrier)
            record_reserved();
        }
        // ---- 5. delivery into this tile's ring ----------------------------------
        if (S == 0 && l == 0) s_paths[kPathNoSpikes] += 1;
        for (int b0 = 0; b0 < S; b0 += kSpkBatch) {
            const int nb = min(kSpkBatch, S - b0);
            // every tile at most kWordIds spikes: the sub-rows are in the pollers'
            // registers (fast); otherwise look them up here
            const bool fast = NPT == 1 && T <= nthr && S <= kSpkBatch && s_many != static_cast<int>(n);
            const bool direct = NPT == 1 && b0 == 0 && T <= nthr && s_big != static_cast<int>(n);
            // spike b0 + q of the step: its id (from its tile's word, or an entry
            // word from the fifth spike of a tile on) and this tile's sub-row of it
            auto subrow_of = [&](int q) {
                const int g = b0 + q;
                int src, k;
                if (direct) {
                    const int v = s_src[g];
                    src = v >> 16;
                    k = v & 0xFFFF;
                } else {
                    src = find_segment(s_cnt, T + 1, g);
                    k = g - s_cnt[src];
                }
                int pre = td.inst_n0 + src * td.stride + word_offset(s_word[src], min(k, kWordIds - 1));
                if (k >= kWordIds) {
                    uint64_t w = 0;
                    if (!wait_word(entries + static_cast<size_t>(src) * tmax + k, P,
                                   [tag32](uint64_t x) { return (x >> 32) == tag32; }, w)) {
                        s_abort = 1;
                        w = static_cast<uint32_t>(td.inst_n0);
                    }
                    pre = static_cast<int>(static_cast<uint32_t>(w));
                }
                return P.subrow[td.sub_base + static_cast<int64_t>(pre - td.inst_n0) * T];
            };
            const bool grouped = fast && !BUDGET && nb * kGroupMin <= nthr;
            // delivery-path counters (the choice is uniform over the workgroup)
            if (l == 0) {
                s_paths[grouped ? kPathGrouped : fast ? kPathFast : nb <= nthr ? kPathPerThread : kPathBatched] += 1;
                if (b0 > 0) s_paths[kPathExtraBatch] += 1;
                if (!fast) s_paths[direct ? kPathDirectMap : kPathSearch] += 1;
                if (s_many == static_cast<int>(n)) s_paths[kPathEntryWords] += 1;
            }
            if (grouped) {
                if (l < T) {
#pragma unroll
                    for (int k = 0; k < kWordIds; ++k)
                        if (k < nk) {
                            s_beg[ex_l + k] = static_cast<int>(sr_first[k].x);
                            s_pre[ex_l + k] = static_cast<int>(sr_first[k].y);
                        }
                }
                __syncthreads();
            } else if (fast) {
                // s_pre: the sub-row lengths, or (step budget) their exclusive prefix
                int run = 0, total = 0;
                if (BUDGET) {
                    int len = 0;
#pragma unroll
                    for (int k = 0; k < kWordIds; ++k)
                        if (k < nk) len += static_cast<int>(sr_first[k].y);
                    run = block_scan_excl(len, s_wave, &total);
                }
#pragma unroll
                for (int k = 0; k < kWordIds; ++k)
                    if (k < nk) {
                        s_beg[ex_l + k] = static_cast<int>(sr_first[k].x);
                        s_pre[ex_l + k] = BUDGET ? run : static_cast<int>(sr_first[k].y);
                        run += static_cast<int>(sr_first[k].y);
                    }
                if (BUDGET && l == 0) s_pre[nb] = total;
                __syncthreads();
            } else if (nb <= nthr) {
                // one spike per thread
                int len = 0;
                if (l < nb) {
                    const uint2 sr = subrow_of(l);
                    s_beg[l] = static_cast<int>(sr.x);
                    len = static_cast<int>(sr.y);
                }
                if (BUDGET) {
                    int total;
                    const int ex = block_scan_excl(len, s_wave, &total);
                    if (l < nb) s_pre[l] = ex;
                    if (l == 0) s_pre[nb] = total;
                } else if (l < nb) {
                    s_pre[l] = len;
                }
                __syncthreads();
                if (s_abort) break;
            } else {
                for (int q = l; q < nb; q += nthr) {
                    const uint2 sr = subrow_of(q);
                    s_beg[q] = static_cast<int>(sr.x);
                    s_pre[q] = static_cast<int>(sr.y);
                }
                __syncthreads();
                if (s_abort) break;
                if (BUDGET) lds_scan_excl(s_pre, nb, s_wave);
            }
            if (tr && b0 == 0) tr[5] = __builtin_amdgcn_s_memrealtime();
            auto add = [&](int tg, int d, int wq) {
                const int ds = static_cast<int>((n + d) & mask);
                if (LRING) {
                    atomicAdd(ring + ds * tmax + tg, wq);
                } else if (d <= W) {
                    int row = wslot + d;
                    if (row >= W) row -= W;
                    atomicAdd(ring + row * tmax + tg, wq);
                } else {
                    __hip_atomic_fetch_add(gring + ds * P.gstride + tg, wq, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            };
            if (grouped) {
                ev_acc += deliver_grouped<SF, kDeliverU>(P.syn, s_beg, s_pre, nb, add);
            } else if (!BUDGET) {
                ev_acc += deliver_cursor<SF, kCursorU>(P.syn, s_beg, s_pre, nb, P.lanes, add);
            } else {
                const int E = s_pre[nb];
                if (l == 0) ev_acc += static_cast<unsigned long long>(E);
                deliver_events<SF, kDeliverU>(P.syn, s_beg, s_pre, nb, E, add, t_step, P.budget_ticks, &drop_acc);
            }
            __syncthreads();
        }
        if (s_abort) break;
        if (tr) tr[6] = __builtin_amdgcn_s_memrealtime();
    }

    if (tr_launch) tr_launch[2] = __builtin_amdgcn_s_memrealtime();
    // ---- write back state, ring and counters -------------------------------------
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = l + k * nthr;
        if (q < tlen) {
            const int32_t i = t0 + q;
            B.u[i] = u[k];
            B.cur[i] = I[k];
            B.refr[i] = static_cast<uint8_t>(r[k]);
        }
    }
    __syncthreads();
    if (tr_launch) tr_launch[4] = __builtin_amdgcn_s_memrealtime();
    // the window rows hold slots n .. n + W - 1 (n: the next step)
    const int n_slot = static_cast<int>(n & mask), n_row = W ? static_cast<int>(n % W) : 0;
    for (int s0 = 0; s0 < R; s0 += kRingBatch)
        for (int q = l; q < tlen; q += nthr) {
            int v[kRingBatch];
#pragma unroll
            for (int k2 = 0; k2 < kRingBatch; ++k2) {
                const int s2 = s0 + k2;
                v[k2] = s2 >= R ? 0 : LRING ? ring[s2 * tmax + q] : gring[s2 * P.gstride + q];
            }
#pragma unroll
            for (int k2 = 0; k2 < kRingBatch; ++k2) {
                const int s2 = s0 + k2;
                if (s2 >= R) continue;
                if (!LRING) {
                    const int k = (s2 - n_slot) & mask;
                    if (k < W) {
                        int row = n_row + k;
                        if (row >= W) row -= W;
                        v[k2] += ring[row * tmax + q];
                    }
                }
                B.ring[static_cast<size_t>(s2) * B.n + t0 + q] = v[k2];
            }
        }
    if (tr_launch) tr_launch[5] = __builtin_amdgcn_s_memrealtime();
    unsigned long long ps = pois_sum, dr = drop_acc, ev = ev_acc;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ps += __shfl_xor(ps, o, 64);
        dr += __shfl_xor(dr, o, 64);
        ev += __shfl_xor(ev, o, 64);
    }
    if ((l & 63) == 0 && ev && !s_abort) atomicAdd(&ctl->events, ev);
    if ((l & 63) == 0 && ps) atomicAdd(&B.pois_acc[t], ps);
    if (BUDGET) {
        if ((l & 63) == 0 && dr) atomicAdd(&s_drop, dr);
        __syncthreads();
    }
    if (tr_launch) tr_launch[6] = __builtin_amdgcn_s_memrealtime();
    if (l == 0)
        for (int k = 0; k < kPaths; ++k)
            if (s_paths[k]) atomicAdd(&P.paths[k], static_cast<unsigned long long>(s_paths[k]));
    if (l == 0) {
        // this launch's counters: the events this tile dropped (every launch
        // writes its own, so nothing is cleared in between) ...
        P.dropped[t] = BUDGET ? s_drop : 0ull;
        if (t == 0) {
            if (!s_abort) ctl->nbase = n;
            if (T == P.n_tiles) P.head->rec_total = static_cast<unsigned long long>(rec_base);
            // ... and the other buffer's counters, zeroed for the next launch
            P.head_other->rec_total = 0;
            P.head_other->flags = 0;
        }
        if (tr_launch) tr_launch[3] = __builtin_amdgcn_s_memrealtime();
    }
}

// Sub-row table: entry (tile t, presynaptic neuron i of t's instance) = first
// synapse and count of the part of row i whose targets lie in tile t (rows are
// sorted by target, so that part is contiguous).
// One thread per presynaptic neuron i: cut its row (sorted by target) at the
// boundaries of its instance's tiles and write the (first, count) pairs of all
// those tiles side by side, entry sub_base(tile) + (i - inst_n0) * T.
__global__ void k_subrows(const uint64_t *row_ptr, const int32_t *tgt, const TileDesc *tiles, int n_tiles,
                          int64_t n_neurons, uint2 *subrow)
{
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= n_neurons) return;
    const int32_t i = static_cast<int32_t>(q);
    int lo = 0, hi = n_tiles;                      // tile holding neuron i: its instance's tiles
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tiles[mid].t0 <= i) lo = mid; else hi = mid;
    }
    const int first = tiles[lo].itile0, T = tiles[lo].intiles;
    const int64_t p = i - tiles[lo].inst_n0;
    uint64_t a = row_ptr[i];
    const uint64_t end = row_ptr[i + 1];
    for (int k = 0; k < T; ++k) {
        const TileDesc td = tiles[first + k];
        const int32_t k1 = td.t0 + td.len;
        uint64_t c = a, e = end;                   // first synapse at or beyond the tile's end
        while (c < e) {
            const uint64_t mid = (c + e) >> 1;
            if (tgt[mid] < k1) c = mid + 1; else e = mid;
        }
        subrow[td.sub_base + p * T] = make_uint2(static_cast<uint32_t>(a), static_cast<uint32_t>(c - a));
        a = c;
    }
}

// Packed record of every synapse (grid-stride over the store).
__global__ void k_pack_synapses(const int32_t *tgt, const uint8_t *dly, const void *w, int wfmt, const TileDesc *tiles,
                                const int32_t *tile_of, int64_t m, int syn_fmt, void *syn)
{
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < m;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t g = tgt[j];
        const uint32_t local = static_cast<uint32_t>(g - tiles[tile_of[g]].t0);
        const uint32_t d = dly[j];
        uint32_t wbits = wfmt == 0 ? __float_as_uint(static_cast<const float *>(w)[j]) : static_cast<const uint16_t *>(w)[j];
        if (syn_fmt <= kSyn8BF16) {
            static_cast<uint2 *>(syn)[j] = make_uint2(local | (d << 16), wbits);
        } else {
            static_cast<uint32_t *>(syn)[j] = local | (d << 10) | (wbits << 16);
        }
    }
}

template <int SF, bool LR, int NPT>
const void *tiled_fn3(int mode)
{
    switch (mode) {
    case 0: return reinterpret_cast<const void *>(&k_tiled<SF, LR, NPT, 0>);
    case 1: return reinterpret_cast<const void *>(&k_tiled<SF, LR, NPT, 1>);
    case 2: return reinterpret_cast<const void *>(&k_tiled<SF, LR, NPT, 2>);
    default: return reinterpret_cast<const void *>(&k_tiled<SF, LR, NPT, 3>);
    }
}

template <int SF, bool LR>
const void *tiled_fn2(int npt, int mode)
{
    return npt == 1 ? tiled_fn3<SF, LR, 1>(mode) : npt == 2 ? tiled_fn3<SF, LR, 2>(mode) : tiled_fn3<SF, LR, 4>(mode);
}

template <int SF>
const void *tiled_fn1(bool lr, int npt, int mode)
{
    return lr ? tiled_fn2<SF, true>(npt, mode) : tiled_fn2<SF, false>(npt, mode);
}

// mode: bit 0 step budget, bit 1 phase trace
const void *tiled_kernel(int sf, bool lr, int npt, int mode)
{
    switch (sf) {
    case kSyn8F32: return tiled_fn1<kSyn8F32>(lr, npt, mode);
    case kSyn8F16: return tiled_fn1<kSyn8F16>(lr, npt, mode);
    case kSyn8BF16: return tiled_fn1<kSyn8BF16>(lr, npt, mode);
    case kSyn4F16: return tiled_fn1<kSyn4F16>(lr, npt, mode);
    default: return tiled_fn1<kSyn4BF16>(lr, npt, mode);
    }
}

}  // namespace

TiledShape tiled_shape(int tile_max, int max_intiles, int ring, bool lds_ring, int win)
{
    TiledShape sh{};
    sh.lds_ring = lds_ring;
    sh.win = lds_ring ? 0 : win;
    sh.npt = tile_max <= 1024 ? 1 : tile_max <= 2048 ? 2 : 4;
    const int per_thread = (tile_max + sh.npt - 1) / sh.npt;
    sh.threads = ((per_thread + 63) / 64) * 64;
    const size_t ring_ints = lds_ring ? static_cast<size_t>(ring) * tile_max : ((static_cast<size_t>(sh.win) * tile_max + 1) & ~size_t{1});
    sh.lds = sizeof(int) * (ring_ints + 16 * (static_cast<size_t>(tile_max) / 8 + 2) +
                            (3 * static_cast<size_t>(max_intiles) + 1) + 2 * kSpkBatch + 1 + tile_max);
    return sh;
}

hipError_t tiled_max_coresident(int syn_fmt, const TiledShape &sh, int *blocks_per_cu)
{
    // every form (step budget, phase trace) must fit
    *blocks_per_cu = 1 << 30;
    for (int mode = 0; mode < 4; ++mode) {
        const void *f = tiled_kernel(syn_fmt, sh.lds_ring, sh.npt, mode);
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sh.lds));
        if (e != hipSuccess) return e;
        int b = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, f, sh.threads, sh.lds);
        if (e != hipSuccess) return e;
        // The occupancy query can count more workgroups per compute unit than
        // their LDS (static + dynamic) leaves room for; a tiling that relied
        // on it would wait for workgroups that are never placed.  Bound it by
        // the LDS directly.
        hipFuncAttributes a{};
        e = hipFuncGetAttributes(&a, f);
        if (e != hipSuccess) return e;
        const size_t per = (sh.lds + a.sharedSizeBytes + kLdsBlock - 1) / kLdsBlock * kLdsBlock;
        b = std::min(b, static_cast<int>(kLdsBytes / per));
        *blocks_per_cu = std::min(*blocks_per_cu, b);
    }
    return hipSuccess;
}

hipError_t launch_subrows(const DevNet &d, const TileDesc *tiles_dev, int n_tiles, int64_t n_neurons, uint2 *subrow,
                          hipStream_t st)
{
    const int64_t blocks = (n_neurons + 255) / 256;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_subrows, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, d.row_ptr, d.tgt, tiles_dev,
                       n_tiles, n_neurons, subrow);
    return hipGetLastError();
}

hipError_t launch_pack_synapses(const DevNet &d, const TileDesc *tiles_dev, const int32_t *tile_of, int64_t m,
                                int syn_fmt, void *syn, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_synapses, dim3(8192), dim3(256), 0, st, d.tgt, d.dly, d.w, d.wfmt, tiles_dev, tile_of, m,
                       syn_fmt, syn);
    return hipGetLastError();
}

hipError_t launch_tiled(const TiledNet &tn, const TiledShape &sh, int64_t steps, bool coop, hipStream_t st)
{
    TiledNet arg = tn;
    int64_t nsteps = steps;
    void *args[] = {&arg, &nsteps};
    const int mode = (tn.budget_ticks != 0 ? 1 : 0) | (tn.trace != nullptr ? 2 : 0);
    const void *f = tiled_kernel(tn.syn_fmt, sh.lds_ring, sh.npt, mode);
    if (coop)
        return hipLaunchCooperativeKernel(f, dim3(tn.n_tiles), dim3(sh.threads), args, static_cast<unsigned>(sh.lds), st);
    return hipLaunchKernel(f, dim3(tn.n_tiles), dim3(sh.threads), args, static_cast<unsigned>(sh.lds), st);
}

}  // namespace mc

// ===========================================================================
// Spike injection: deliver the synaptic rows of a given list of neurons as if
// they had spiked in the step before `n` (their weights land in slots
// (n - 1 + d) mod R).  Used for external stimulation and to measure delivery on
// large spike lists.
// ===========================================================================
namespace mc {
namespace {

// One workgroup per tile: gather the tile's sub-rows of all listed neurons,
// accumulate into an LDS copy of the tile's ring, then add it into the ring.
// Tiles are taken XCD by XCD (as in the step kernel), so that the sub-rows of
// one neuron that neighbouring tiles read, and their entries, share lines in
// one L2: taken in launch order, every XCD would fetch every line of a row.
template <int SF>
__global__ __launch_bounds__(1024) void k_inject_tiled(TiledNet P, const int32_t *ids, int32_t count, int32_t id_offset,
                                                       int64_t n, int batch)
{
    extern __shared__ int lds[];
    const DevNet &B = P.base;
    const int t = xcd_tile(blockIdx.x, gridDim.x) + P.tile_offset;   // tiles of one instance, XCD by XCD
    const TileDesc td = P.tiles[t];
    const int l = threadIdx.x, nthr = blockDim.x;
    const int mask = B.ring_mask, R = mask + 1;
    const int tmax = P.tile_max, tlen = td.len;
    int *ring = lds;                                  // [R][tmax]
    // [batch] (first record, length) of each spike's sub-row, 8-byte aligned
    int2 *s_row = reinterpret_cast<int2 *>(ring + ((R * tmax + 1) & ~1));
    for (int q = l; q < R * tmax; q += nthr) ring[q] = 0;
    __syncthreads();
    for (int b0 = 0; b0 < count; b0 += batch) {
        const int nb = min(batch, count - b0);
        for (int q = l; q < nb; q += nthr) {
            const uint2 sr = P.subrow[td.sub_base + static_cast<int64_t>(ids[b0 + q] + id_offset - td.inst_n0) * td.intiles];
            s_row[q] = make_int2(static_cast<int>(sr.x), static_cast<int>(sr.y));
        }
        __syncthreads();
        deliver_chunks_pipelined<SF, kInjectU>(P.syn, s_row, nb, P.lanes, [&](int tg, int d, int wq) {
            atomicAdd(ring + static_cast<int>((n - 1 + d) & mask) * tmax + tg, wq);
        });
        __syncthreads();
    }
    // add the staged ring into the global one: the tile's R x tlen cells dealt
    // to all threads in order (coalesced within a slot), kInjWriteBack cells'
    // loads in flight per thread; cells that received nothing are left alone.
    // Thread l's cells are c = l + j nthr, walked as (slot, neuron) pairs.
    const int cells = R * tlen, ds = nthr / tlen, dq = nthr - ds * tlen;
    int slot = l / tlen, q = l - slot * tlen;
    for (int c0 = 0; c0 < cells; c0 += kInjWriteBack * nthr) {
        int v[kInjWriteBack], g[kInjWriteBack], s_k[kInjWriteBack], q_k[kInjWriteBack];
#pragma unroll
        for (int k = 0; k < kInjWriteBack; ++k) {
            s_k[k] = slot;
            q_k[k] = q;
            v[k] = slot < R ? ring[slot * tmax + q] : 0;
            g[k] = v[k] ? B.ring[static_cast<int64_t>(slot) * B.n + td.t0 + q] : 0;
            slot += ds;
            q += dq;
            if (q >= tlen) {
                q -= tlen;
                ++slot;
            }
        }
#pragma unroll
        for (int k = 0; k < kInjWriteBack; ++k)
            if (v[k]) B.ring[static_cast<int64_t>(s_k[k]) * B.n + td.t0 + q_k[k]] = g[k] + v[k];
    }
}

// Fallback: one wavefront per listed neuron's row chunk of `seg` synapses,
// device-scope int32 atomics into the global ring.
template <int WF>
__global__ __launch_bounds__(256) void k_inject_global(DevNet P, const int32_t *ids, int32_t count, int32_t id_offset,
                                                      int64_t n)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * 4;
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); w < count; w += waves) {
        const int32_t pre = ids[w] + id_offset;
        const uint64_t j0 = P.row_ptr[pre], j1 = P.row_ptr[pre + 1];
        for (uint64_t j = j0 + lane; j < j1; j += 64) {
            const int d = P.dly[j];
            atomicAdd(P.ring + static_cast<size_t>((n - 1 + d) & P.ring_mask) * P.n + P.tgt[j], weight_q8<WF>(P.w, j));
        }
    }
}

template <int SF>
const void *inject_tiled_fn() { return reinterpret_cast<const void *>(&k_inject_tiled<SF>); }

}  // namespace

int inject_batch(int tile_max, int ring)
{
    const size_t ring_bytes = sizeof(int) * (static_cast<size_t>(ring) * tile_max + 1) + 256;
    if (ring_bytes >= kLdsBytes) return 0;
    const size_t fit = (kLdsBytes - ring_bytes) / (2 * sizeof(int)) / 256 * 256;
    return static_cast<int>(std::min<size_t>(kInjBatchMax, fit));
}

size_t inject_lds_bytes(int tile_max, int ring)
{
    return sizeof(int) * (static_cast<size_t>(ring) * tile_max + 2 * static_cast<size_t>(inject_batch(tile_max, ring)) + 1);
}

hipError_t launch_inject_tiled(const TiledNet &tn, int first_tile, int ntiles, int threads, const int32_t *ids,
                               int32_t count, int32_t id_offset, int64_t n, hipStream_t st)
{
    TiledNet arg = tn;
    arg.tile_offset = first_tile;
    const int batch = inject_batch(tn.tile_max, tn.base.ring_mask + 1);
    if (batch <= 0) return hipErrorInvalidValue;
    const size_t lds = inject_lds_bytes(tn.tile_max, tn.base.ring_mask + 1);
    const void *f = tn.syn_fmt == kSyn8F32 ? inject_tiled_fn<kSyn8F32>()
                  : tn.syn_fmt == kSyn8F16 ? inject_tiled_fn<kSyn8F16>()
                  : tn.syn_fmt == kSyn8BF16 ? inject_tiled_fn<kSyn8BF16>()
                  : tn.syn_fmt == kSyn4F16 ? inject_tiled_fn<kSyn4F16>() : inject_tiled_fn<kSyn4BF16>();
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    int batch_arg = batch;
    void *args[] = {&arg, const_cast<int32_t **>(&ids), &count, &id_offset, &n, &batch_arg};
    return hipLaunchKernel(f, dim3(ntiles), dim3(threads), args, lds, st);
}

hipError_t launch_inject_global(const DevNet &d, const int32_t *ids, int32_t count, int32_t id_offset, int64_t n,
                                hipStream_t st)
{
    const int blocks = static_cast<int>(std::min<int64_t>(4096, (static_cast<int64_t>(count) + 3) / 4));
    if (blocks < 1) return hipSuccess;
    switch (d.wfmt) {
    case 0: hipLaunchKernelGGL(k_inject_global<0>, dim3(blocks), dim3(256), 0, st, d, ids, count, id_offset, n); break;
    case 1: hipLaunchKernelGGL(k_inject_global<1>, dim3(blocks), dim3(256), 0, st, d, ids, count, id_offset, n); break;
    default: hipLaunchKernelGGL(k_inject_global<2>, dim3(blocks), dim3(256), 0, st, d, ids, count, id_offset, n); break;
    }
    return hipGetLastError();
}

}  // namespace mc
