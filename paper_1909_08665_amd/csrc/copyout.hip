// copyout.hip -- the recorder's way back to the host: after each launch of the
// step kernel, a small kernel copies the recorder head and the first entries
// into pinned host memory (the launch's spikes, Sec. 3a(ii) recording).  It
// starts sooner after the step kernel than the runtime's device-to-host copy
// does, so a short mc_run returns sooner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"

namespace mc {
namespace {

// Copy a recorder's head and its first min(rec_total, n) entries into pinned
// host memory (grid-stride; the launch that filled the recorder ran before it
// on the same stream).
__global__ __launch_bounds__(1024) void k_copy_out(const RecHead *head, const uint64_t *rec, int64_t n,
                                                   RecHead *h_head, uint64_t *h_rec)
{
    const unsigned long long total = head->rec_total;
    const int64_t cnt = min(static_cast<int64_t>(total), n);
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < cnt;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x)
        h_rec[q] = rec[q];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        h_head->rec_total = total;
        h_head->flags = head->flags;
    }
}

}  // namespace

hipError_t launch_copy_out(const RecHead *head, const uint64_t *rec, int64_t n, RecHead *h_head, uint64_t *h_rec,
                           hipStream_t st)
{
    const int64_t per_block = 8192;
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(64, std::max<int64_t>(1, (n + per_block - 1) / per_block)));
    hipLaunchKernelGGL(k_copy_out, dim3(blocks), dim3(1024), 0, st, head, rec, n, h_head, h_rec);
    return hipGetLastError();
}

}  // namespace mc
