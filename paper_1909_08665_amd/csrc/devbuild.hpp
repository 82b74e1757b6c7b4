// devbuild.hpp -- construction of the synapse store on the GPU.
//
// The same draw as the host builder (Sec. 2a of Rhodes et al., arXiv
// 1909.08665: fixed-total pairwise connectivity, normal weights and delays;
// Philox4x64-10 counter (index within the pair, 8a + b, 0, 1), key (seed, 0);
// Box-Muller on words 2 and 3), run one thread per synapse, then the CSR row
// order (presynaptic neuron; within a row target, delay, weight) by two stable
// radix sorts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "model.hpp"

namespace mc {

// Fills row_ptr [N+1], tgt [M], dly [M] and w [M] (float holding wq / 256 for
// the FP32 store, FP16/BF16 bits otherwise) for the network planned in H and
// segs, on stream st.  On success sets max_d (largest delay) and max_in_abs
// (largest sum over a neuron's incoming synapses of |wq|), and returns 0;
// otherwise an MC_ERR_* code with msg set.  Needs N < 2^24 (the target id
// shares a 64-bit sort key with the delay and the weight).  Scratch: about
// 42 bytes per synapse, freed before returning.
int build_synapses_on_device(const ModelParams &p, const HostNet &H, const std::vector<SynSeg> &segs,
                             uint64_t *row_ptr, int32_t *tgt, uint8_t *dly, void *w, hipStream_t st, int &max_d,
                             int64_t &max_in_abs, std::string &msg);

}  // namespace mc
