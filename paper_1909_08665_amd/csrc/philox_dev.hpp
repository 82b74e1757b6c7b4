// philox_dev.hpp -- Philox4x64-10 (Salmon et al., SC'11) on the GPU: ten rounds
// of two 64 x 64 -> 128-bit products, round keys bumped by the Weyl constants.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mc {

// Block for counter (c0, c1, c2, c3), key (seed, 0).
__device__ __forceinline__ void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t seed,
                                           uint64_t out[4])
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL, kMulB = 0xCA5A826395121157ULL;
    constexpr uint64_t kBumpA = 0x9E3779B97F4A7C15ULL, kBumpB = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
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
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

}  // namespace mc
