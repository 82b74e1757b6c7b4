// probe.hip -- ceilings of the memory system the step kernels run against,
// measured on the device at hand: streaming HBM bandwidth, the rate of LDS
// integer atomics (the tiled engine's ring updates) and the rate of device
// integer atomics on random targets in a buffer of a chosen size (resident in
// L2, in the Infinity Cache, or spread over HBM: the global-ring variants and
// the graph engine's delivery), and the rate of whole cache-line reads at
// random places of a large buffer (what sub-row reads at random places cost
// HBM, which no streaming copy shows).  Each probe times its kernel with HIP events
// on a stream of its own and returns the rate.
#include <hip/hip_runtime.h>

#include <cstdint>
#include "kernels.hpp"

namespace mc {
namespace {

// Per-thread pseudo-random stream (a 32-bit linear congruential generator
// seeded by a hash of the thread index): addresses spread over the target.
__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t lcg(uint32_t x) { return x * 1664525U + 1013904223U; }

constexpr int kProbeThreads = 1024;
constexpr int kLdsWords = 16384;             // 64 KB of LDS per workgroup

// LDS atomics: every thread adds 1 at `iters` random words of the
// workgroup's LDS array, then the array's sum is written out (it must equal
// threads x iters, which also keeps the adds from being optimised away).
__global__ __launch_bounds__(kProbeThreads) void k_probe_lds_atomics(uint32_t iters, unsigned long long *sums)
{
    __shared__ uint32_t a[kLdsWords];
    for (int q = threadIdx.x; q < kLdsWords; q += blockDim.x) a[q] = 0;
    __syncthreads();
    uint32_t x = mix(blockIdx.x * blockDim.x + threadIdx.x + 1);
    for (uint32_t i = 0; i < iters; ++i) {
        x = lcg(x);
        atomicAdd(&a[(x >> 8) & (kLdsWords - 1)], 1u);
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int q = threadIdx.x; q < kLdsWords; q += blockDim.x) s += a[q];
    atomicAdd(&sums[blockIdx.x], s);
}

// Device atomics: every thread adds 1 at `iters` random words of a buffer of
// mask + 1 words (a power of two); the results are not returned (the form the
// delivery kernels use).
__global__ __launch_bounds__(256) void k_probe_global_atomics(uint32_t *buf, uint64_t mask, uint32_t iters)
{
    uint64_t x = mix(blockIdx.x * blockDim.x + threadIdx.x + 1);
    uint64_t y = mix(static_cast<uint32_t>(x) ^ 0x9e3779b9U);
    for (uint32_t i = 0; i < iters; ++i) {
        x = lcg(static_cast<uint32_t>(x));
        y = lcg(static_cast<uint32_t>(y));
        const uint64_t at = ((x << 32) | y) & mask;
        atomicAdd(&buf[at], 1u);
    }
}

// Gather: lanes in groups of 16 read one 128-byte cache line (8 bytes each)
// at random line-aligned places of a buffer of mask + 1 lines -- the unit in
// which a sub-row read at a random place reaches HBM (every L2 miss fetches a
// whole line) -- 8 reads in flight per lane, for `rounds` rounds; the xor of
// what a thread read is stored, so that no read can be dropped.
constexpr int kGatherU = 8;
constexpr int kGatherLanes = 16;
__global__ __launch_bounds__(kProbeThreads) void k_probe_gather(const uint2 *__restrict__ buf, uint64_t mask,
                                                                uint32_t rounds, uint2 *out)
{
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = id % kGatherLanes, g = id / kGatherLanes;   // the group's lanes draw the same places
    uint32_t x = mix(g + 1), y = mix(g ^ 0x9e3779b9U);
    uint2 acc = make_uint2(0u, 0u);
    for (uint32_t i = 0; i < rounds; ++i) {
        uint2 v[kGatherU];
#pragma unroll
        for (int k = 0; k < kGatherU; ++k) {
            x = lcg(x);
            y = lcg(y);
            const uint64_t c = ((static_cast<uint64_t>(x) << 32) | y) & mask;
            v[k] = buf[c * kGatherLanes + r];
        }
#pragma unroll
        for (int k = 0; k < kGatherU; ++k) {
            acc.x ^= v[k].x;
            acc.y ^= v[k].y;
        }
    }
    out[id] = acc;
}

// Streaming copy, 16 bytes per load and store, grid-stride.
__global__ __launch_bounds__(256) void k_probe_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n)
{
    for (uint64_t q = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
         q += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        dst[q] = src[q];
}

}  // namespace

hipError_t run_probe(int kind, int64_t bytes, double *rate, double *kernel_ms)
{
    *rate = 0.0;
    *kernel_ms = 0.0;
    int dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *a = nullptr, *b = nullptr;
    double work = 0.0;                       // bytes moved or atomics done by one timed launch
    auto ok = [&err](hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
        return err == hipSuccess;
    };
    if (ok(hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) && ok(hipEventCreate(&e0)) && ok(hipEventCreate(&e1))) {
        if (kind == kProbeHbmCopy) {
            const uint64_t half = static_cast<uint64_t>(bytes) / 2 / sizeof(uint4);
            if (ok(hipMalloc(&a, half * sizeof(uint4))) && ok(hipMalloc(&b, half * sizeof(uint4))) &&
                ok(hipMemsetAsync(a, 1, half * sizeof(uint4), st))) {
                const int grid = cus * 16;
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {      // the first launch warms up
                    ok(hipEventRecord(e0, st));
                    hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, st, static_cast<const uint4 *>(a),
                                       static_cast<uint4 *>(b), half);
                    ok(hipGetLastError());
                    ok(hipEventRecord(e1, st));
                }
                work = 2.0 * static_cast<double>(half * sizeof(uint4));
            }
        } else if (kind == kProbeLdsAtomics) {
            const int grid = cus * 2;                                       // two 1024-thread workgroups per CU
            const uint32_t iters = 4096;
            if (ok(hipMalloc(&a, grid * sizeof(unsigned long long)))) {
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
                    ok(hipMemsetAsync(a, 0, grid * sizeof(unsigned long long), st));
                    ok(hipEventRecord(e0, st));
                    hipLaunchKernelGGL(k_probe_lds_atomics, dim3(grid), dim3(kProbeThreads), 0, st, iters,
                                       static_cast<unsigned long long *>(a));
                    ok(hipGetLastError());
                    ok(hipEventRecord(e1, st));
                }
                work = static_cast<double>(grid) * kProbeThreads * iters;
                // every add must have landed
                unsigned long long first = 0;
                if (ok(hipStreamSynchronize(st)) && ok(hipMemcpy(&first, a, sizeof(first), hipMemcpyDeviceToHost)) &&
                    first != static_cast<unsigned long long>(kProbeThreads) * iters)
                    err = hipErrorUnknown;
            }
        } else if (kind == kProbeHbmGather) {
            uint64_t chunks = 64;                                           // 128-byte lines, a power of two
            while (chunks * 2 * 128 <= static_cast<uint64_t>(bytes)) chunks *= 2;
            const int grid = cus * 2;                                       // two 1024-thread workgroups per CU
            const uint32_t rounds = 64;
            if (ok(hipMalloc(&a, chunks * 128)) && ok(hipMemsetAsync(a, 3, chunks * 128, st)) &&
                ok(hipMalloc(&b, static_cast<size_t>(grid) * kProbeThreads * sizeof(uint2)))) {
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
                    ok(hipEventRecord(e0, st));
                    hipLaunchKernelGGL(k_probe_gather, dim3(grid), dim3(kProbeThreads), 0, st,
                                       static_cast<const uint2 *>(a), chunks - 1, rounds, static_cast<uint2 *>(b));
                    ok(hipGetLastError());
                    ok(hipEventRecord(e1, st));
                }
                work = static_cast<double>(grid) * kProbeThreads * rounds * kGatherU * sizeof(uint2);
            }
        } else {
            uint64_t words = 1024;
            while (words * 2 * sizeof(uint32_t) <= static_cast<uint64_t>(bytes)) words *= 2;
            const int grid = cus * 8;
            const uint32_t iters = 256;
            if (ok(hipMalloc(&a, words * sizeof(uint32_t))) && ok(hipMemsetAsync(a, 0, words * sizeof(uint32_t), st))) {
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
                    ok(hipEventRecord(e0, st));
                    hipLaunchKernelGGL(k_probe_global_atomics, dim3(grid), dim3(256), 0, st, static_cast<uint32_t *>(a),
                                       words - 1, iters);
                    ok(hipGetLastError());
                    ok(hipEventRecord(e1, st));
                }
                work = static_cast<double>(grid) * 256 * iters;
            }
        }
        float ms = 0.f;
        if (ok(hipEventSynchronize(e1)) && ok(hipEventElapsedTime(&ms, e0, e1)) && ms > 0.f) {
            const bool bytes_rate = kind == kProbeHbmCopy || kind == kProbeHbmGather;
            *rate = bytes_rate ? work / (ms * 1e-3) / 1e9 : work / (ms * 1e-3);
            *kernel_ms = ms;
        }
    }
    if (st) hipStreamSynchronize(st);
    if (a) hipFree(a);
    if (b) hipFree(b);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (st) hipStreamDestroy(st);
    return err;
}

}  // namespace mc
