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
#include "kernels.hpp"

namespace mc {
namespace {

constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL, kMulB = 0xCA5A826395121157ULL;
constexpr uint64_t kBumpA = 0x9E3779B97F4A7C15ULL, kBumpB = 0xBB67AE8584CAA73BULL;

// First output word of Philox4x64-10 for counter (c0, c1, 0, tag), key (seed, 0).
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t tag, uint64_t seed)
{
    uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = tag;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a_lo = kMulA * x0, a_hi = __umul64hi(kMulA, x0);
        const uint64_t b_lo = kMulB * x2, b_hi = __umul64hi(kMulB, x2);
        const uint64_t y0 = b_hi ^ x1 ^ k0;
        const uint64_t y2 = a_hi ^ x3 ^ k1;
        x0 = y0; x1 = b_lo; x2 = y2; x3 = a_lo;
        k0 += kBumpA; k1 += kBumpB;
    }
    return x0;
}

// Background spikes of neuron `local` at step n: the number of CDF thresholds
// not above a 32-bit uniform (inversion of the Poisson distribution).
__device__ __forceinline__ int poisson_draw(uint64_t seed, int64_t n, int32_t local, const uint64_t *thr)
{
    const uint64_t v = philox_word0(static_cast<uint64_t>(n), static_cast<uint64_t>(local), 2, seed) >> 32;
    int k = 0;
    while (k < kPoisMaxDev && v >= thr[k]) ++k;
    return k;
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
                P.rec_id[pos] = i;
                P.rec_step[pos] = static_cast<int32_t>(n);
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
