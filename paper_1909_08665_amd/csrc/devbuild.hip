// devbuild.hip -- the synapse store built on the GPU (see devbuild.hpp).
//
// Per synapse s of pair (a -> b) of an instance (Sec. 2a of Rhodes et al.,
// arXiv 1909.08665): one Philox4x64-10 block x for counter (s - first, 8a + b,
// 0, 1), key (seed, 0); pre and post uniform in a and b from words 0 and 1
// (floor(x * N / 2^64)); a normal pair by Box-Muller from words 2 and 3, the
// first for the weight (mean, sd by source class; clipped at zero on the
// wrong side, Dale's law), the second for the delay (rounded to the step,
// clipped to [1, 255], the 255-slot buffer of Sec. 3a(ii)); the weight rounded
// to the store's format and to units of 1/256 pA.
//
// Every operation is the IEEE double operation the host builder performs
// (no fused multiply-add); log, sqrt, cos and sin are the device library's.
// Their results can differ from the host's in the last place, which changes a
// quantised weight or delay only when the exact value lies within about 1e-13
// of a rounding boundary.
//
// Row order: a stable radix sort by the 64-bit key (target, delay, weight),
// then a stable radix sort by presynaptic neuron, gives rows sorted by
// (target, delay, weight) -- the host builder's order.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>

#include "../../include/mc.h"
#include "devbuild.hpp"
#include "philox_dev.hpp"

namespace mc {
namespace {

// One (instance, pair) segment with everything its draws need.
struct DevSeg {
    int64_t first, count;
    uint64_t seed;
    int32_t pre0, npre, post0, npost;
    int32_t pair, excitatory;
    double mean, sd, dmean, dsd;
};

// Round-to-nearest-even from double to a binary format with `frac` fraction
// bits, exponent bias `bias` and all-ones exponent field `emax_field`: the
// bit pattern.  Exact operations only (ilogb, ldexp, rint).
__device__ uint16_t round_format_bits(double x, int frac, int bias, int emax_field)
{
    const int exp_bits = emax_field == 31 ? 5 : 8;
    const uint16_t sign = signbit(x) ? static_cast<uint16_t>(1u << (frac + exp_bits)) : 0;
    const double a = fabs(x);
    if (a == 0.0) return sign;
    int e = ilogb(a);
    const int emin = 1 - bias;
    if (e < emin) return static_cast<uint16_t>(sign | static_cast<uint16_t>(rint(ldexp(a, frac - emin))));
    double m = rint(ldexp(a, frac - e));
    if (m == ldexp(1.0, frac + 1)) {
        m = ldexp(1.0, frac);
        e += 1;
    }
    const int field = e + bias;
    if (field >= emax_field) return static_cast<uint16_t>(sign | (emax_field << frac));
    return static_cast<uint16_t>(sign | (field << frac) | (static_cast<int>(m) - (1 << frac)));
}

__device__ double format_value(uint16_t h, int wfmt)
{
    if (wfmt == kWFp16) {
        const int f = (h >> 10) & 31, m = h & 1023;
        const double v = f == 0 ? ldexp(static_cast<double>(m), -24) : ldexp(static_cast<double>(1024 + m), f - 25);
        return (h >> 15) ? -v : v;
    }
    return static_cast<double>(__uint_as_float(static_cast<uint32_t>(h) << 16));
}

// Draw synapse s: presynaptic id into pre[s], (target << 40 | delay << 32 |
// wq + 2^31) into key[s], the 16-bit weight bits into w16[s] (reduced stores).
__global__ void k_draw(const DevSeg *segs, int nseg, int64_t m, double dt_ms, int wfmt, uint32_t *pre, uint64_t *key,
                       uint16_t *w16, int32_t *bad)
{
    constexpr double kTwoPi = 6.283185307179586;
    for (int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < m;
         s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int lo = 0, hi = nseg;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (segs[mid].first <= s) lo = mid; else hi = mid;
        }
        const DevSeg g = segs[lo];
        uint64_t x[4];
        philox4x64(static_cast<uint64_t>(s - g.first), static_cast<uint64_t>(g.pair), 0, kTagSyn, g.seed, x);
        const int32_t p = g.pre0 + static_cast<int32_t>(__umul64hi(x[0], static_cast<uint64_t>(g.npre)));
        const int32_t q = g.post0 + static_cast<int32_t>(__umul64hi(x[1], static_cast<uint64_t>(g.npost)));
        const double u_low = static_cast<double>((x[2] >> 11) + 1) * 0x1p-53;     // (0, 1]
        const double u_high = static_cast<double>(x[3] >> 11) * 0x1p-53;         // [0, 1)
        const double radius = sqrt(-2.0 * log(u_low));
        const double angle = kTwoPi * u_high;
        const double z_w = radius * cos(angle);
        const double z_d = radius * sin(angle);
        double wv = g.mean + g.sd * z_w;
        if (g.excitatory) wv = wv < 0.0 ? 0.0 : wv; else wv = 0.0 < wv ? 0.0 : wv;
        double dsteps = rint((g.dmean + g.dsd * z_d) / dt_ms);
        dsteps = dsteps < 1.0 ? 1.0 : dsteps;
        dsteps = 255.0 < dsteps ? 255.0 : dsteps;
        double stored = wv;
        uint16_t bits = 0;
        if (wfmt == kWFp16) {
            bits = round_format_bits(wv, 10, 15, 31);
            stored = format_value(bits, wfmt);
        } else if (wfmt == kWBf16) {
            bits = round_format_bits(wv, 7, 127, 255);
            stored = format_value(bits, wfmt);
        }
        const double wq = rint(stored * 256.0);
        if (!(fabs(wq) < 16777216.0)) atomicOr(bad, 1);
        const uint32_t biased = static_cast<uint32_t>(static_cast<int32_t>(wq)) + 0x80000000u;
        pre[s] = static_cast<uint32_t>(p);
        key[s] = (static_cast<uint64_t>(static_cast<uint32_t>(q)) << 40) | (static_cast<uint64_t>(dsteps) << 32) | biased;
        if (w16) w16[s] = bits;
    }
}

__global__ void k_iota(uint32_t *v, int64_t m)
{
    for (int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < m;
         s += static_cast<int64_t>(gridDim.x) * blockDim.x)
        v[s] = static_cast<uint32_t>(s);
}

__global__ void k_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, int64_t m)
{
    for (int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < m;
         s += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[s] = src[idx[s]];
}

// Final store in row order, the largest delay and every neuron's sum of |wq|.
__global__ void k_emit(const uint64_t *key, const uint16_t *w16, const uint32_t *perm, int64_t m, int wfmt,
                       int32_t *tgt, uint8_t *dly, void *w, int32_t *max_d, unsigned long long *in_abs)
{
    int md = 1;
    for (int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < m;
         s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint32_t o = perm[s];
        const uint64_t k = key[o];
        const int32_t t = static_cast<int32_t>(k >> 40);
        const int d = static_cast<int>((k >> 32) & 0xFFu);
        const int32_t wq = static_cast<int32_t>(static_cast<uint32_t>(k) - 0x80000000u);
        tgt[s] = t;
        dly[s] = static_cast<uint8_t>(d);
        if (wfmt == kWFp32) static_cast<float *>(w)[s] = static_cast<float>(wq) * 0.00390625f;
        else static_cast<uint16_t *>(w)[s] = w16[o];
        md = max(md, d);
        atomicAdd(&in_abs[t], static_cast<unsigned long long>(wq < 0 ? -static_cast<int64_t>(wq) : wq));
    }
    atomicMax(max_d, md);
}

// row_ptr[i] = number of synapses whose presynaptic neuron is below i.
__global__ void k_row_ptr(const uint32_t *pre_sorted, int64_t m, int64_t n, uint64_t *row_ptr)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (static_cast<int64_t>(pre_sorted[mid]) < i) lo = mid + 1; else hi = mid;
    }
    row_ptr[i] = static_cast<uint64_t>(lo);
}

__global__ void k_max_u64(const unsigned long long *v, int64_t n, unsigned long long *out)
{
    unsigned long long mx = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        mx = max(mx, v[i]);
    atomicMax(out, mx);
}

// Device scratch released on every return path.
struct Scratch {
    std::vector<void *> p;
    template <class T>
    hipError_t get(T **out, size_t count)
    {
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(1, count * sizeof(T)));
        if (e == hipSuccess) p.push_back(q);
        *out = static_cast<T *>(q);
        return e;
    }
    ~Scratch()
    {
        for (void *q : p) (void)hipFree(q);
    }
};

}  // namespace

int build_synapses_on_device(const ModelParams &p, const HostNet &H, const std::vector<SynSeg> &segs,
                             uint64_t *row_ptr, int32_t *tgt, uint8_t *dly, void *w, hipStream_t st, int &max_d,
                             int64_t &max_in_abs, std::string &msg)
{
    const int64_t n = H.n, m = H.m;
    if (n >= (int64_t{1} << 24)) {
        msg = "device build needs fewer than 2^24 neurons";
        return MC_ERR_UNSUPPORTED;
    }
    if (m >= (int64_t{1} << 32)) {
        msg = "device build needs fewer than 2^32 synapses";
        return MC_ERR_UNSUPPORTED;
    }
    std::vector<DevSeg> ds;
    for (const SynSeg &g : segs) {
        const int32_t *po = &H.pop_off[static_cast<size_t>(g.inst) * (kPops + 1)];
        DevSeg d{};
        d.first = g.first;
        d.count = g.count;
        d.seed = H.seeds[g.inst];
        d.pre0 = po[g.a];
        d.npre = po[g.a + 1] - po[g.a];
        d.post0 = po[g.b];
        d.npost = po[g.b + 1] - po[g.b];
        d.pair = 8 * g.a + g.b;
        d.excitatory = (g.a % 2) == 0;
        d.mean = d.excitatory ? p.w_mean_pa : p.g * p.w_mean_pa;
        d.sd = d.excitatory ? p.w_sd_pa : std::fabs(p.g) * p.w_sd_pa;
        if (g.a == 2 && g.b == 0) d.mean = p.l4e_l23e_factor * p.w_mean_pa;
        d.dmean = d.excitatory ? p.d_mean_exc_ms : p.d_mean_inh_ms;
        d.dsd = d.excitatory ? p.d_sd_exc_ms : p.d_sd_inh_ms;
        ds.push_back(d);
    }
    auto hip_fail = [&msg](hipError_t e, const char *what) {
        msg = std::string("device build, ") + what + ": " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? MC_ERR_NOMEM : MC_ERR_HIP;
    };
#define DB_TRY(expr, what)                          \
    do {                                            \
        const hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)
    const bool reduced = p.wfmt != kWFp32;
    Scratch sc;
    DevSeg *segs_dev = nullptr;
    uint32_t *pre = nullptr, *iota = nullptr, *perm1 = nullptr, *pre1 = nullptr, *pre2 = nullptr, *perm2 = nullptr;
    uint64_t *key = nullptr, *key_tmp = nullptr;
    uint16_t *w16 = nullptr;
    int32_t *flags = nullptr;     // [0] bad weight, [1] largest delay
    unsigned long long *in_abs = nullptr, *in_max = nullptr;
    DB_TRY(sc.get(&segs_dev, ds.size()), "scratch");
    DB_TRY(sc.get(&pre, m), "scratch");
    DB_TRY(sc.get(&key, m), "scratch");
    DB_TRY(sc.get(&key_tmp, m), "scratch");
    DB_TRY(sc.get(&iota, m), "scratch");
    DB_TRY(sc.get(&perm1, m), "scratch");
    DB_TRY(sc.get(&pre1, m), "scratch");
    DB_TRY(sc.get(&pre2, m), "scratch");
    DB_TRY(sc.get(&perm2, m), "scratch");
    if (reduced) DB_TRY(sc.get(&w16, m), "scratch");
    DB_TRY(sc.get(&flags, 2), "scratch");
    DB_TRY(sc.get(&in_abs, n), "scratch");
    DB_TRY(sc.get(&in_max, 1), "scratch");
    DB_TRY(hipMemcpyAsync(segs_dev, ds.data(), ds.size() * sizeof(DevSeg), hipMemcpyHostToDevice, st), "upload");
    const int32_t init_flags[2] = {0, 1};
    DB_TRY(hipMemcpyAsync(flags, init_flags, sizeof(init_flags), hipMemcpyHostToDevice, st), "upload");
    DB_TRY(hipMemsetAsync(in_abs, 0, std::max<int64_t>(1, n) * sizeof(unsigned long long), st), "clear");
    DB_TRY(hipMemsetAsync(in_max, 0, sizeof(unsigned long long), st), "clear");
    const unsigned grid = 8192, block = 256;
    if (m > 0) {
        hipLaunchKernelGGL(k_draw, dim3(grid), dim3(block), 0, st, segs_dev, static_cast<int>(ds.size()), m, p.dt_ms,
                           p.wfmt, pre, key, w16, flags);
        DB_TRY(hipGetLastError(), "draw");
        hipLaunchKernelGGL(k_iota, dim3(grid), dim3(block), 0, st, iota, m);
        DB_TRY(hipGetLastError(), "draw");
        // (target, delay, weight) over all 64 bits, then presynaptic id: both stable
        const unsigned um = static_cast<unsigned>(m);
        unsigned pre_bits = 1;
        while ((int64_t{1} << pre_bits) <= n) ++pre_bits;
        size_t tb1 = 0, tb2 = 0;
        DB_TRY(rocprim::radix_sort_pairs(nullptr, tb1, key, key_tmp, iota, perm1, um, 0, 64, st), "sort size");
        DB_TRY(rocprim::radix_sort_pairs(nullptr, tb2, pre1, pre2, perm1, perm2, um, 0, pre_bits, st), "sort size");
        void *temp = nullptr;
        DB_TRY(sc.get(reinterpret_cast<uint8_t **>(&temp), std::max(tb1, tb2)), "sort scratch");
        DB_TRY(rocprim::radix_sort_pairs(temp, tb1, key, key_tmp, iota, perm1, um, 0, 64, st), "sort");
        hipLaunchKernelGGL(k_gather_u32, dim3(grid), dim3(block), 0, st, pre, perm1, pre1, m);
        DB_TRY(hipGetLastError(), "gather");
        DB_TRY(rocprim::radix_sort_pairs(temp, tb2, pre1, pre2, perm1, perm2, um, 0, pre_bits, st), "sort");
        hipLaunchKernelGGL(k_emit, dim3(grid), dim3(block), 0, st, key, w16, perm2, m, p.wfmt, tgt, dly, w, flags + 1,
                           in_abs);
        DB_TRY(hipGetLastError(), "emit");
    }
    hipLaunchKernelGGL(k_row_ptr, dim3(static_cast<unsigned>((n + 1 + 255) / 256)), dim3(256), 0, st, pre2, m, n, row_ptr);
    DB_TRY(hipGetLastError(), "row pointers");
    hipLaunchKernelGGL(k_max_u64, dim3(1024), dim3(256), 0, st, in_abs, n, in_max);
    DB_TRY(hipGetLastError(), "bound");
    int32_t hf[2] = {0, 1};
    unsigned long long hmax = 0;
    DB_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st), "download");
    DB_TRY(hipMemcpyAsync(&hmax, in_max, sizeof(hmax), hipMemcpyDeviceToHost, st), "download");
    DB_TRY(hipStreamSynchronize(st), "synchronise");
#undef DB_TRY
    if (hf[0]) {
        msg = "a weight exceeds the 2^24/256 pA range of the fixed-point store";
        return MC_ERR_ARG;
    }
    max_d = hf[1];
    max_in_abs = static_cast<int64_t>(hmax);
    return MC_OK;
}

}  // namespace mc
