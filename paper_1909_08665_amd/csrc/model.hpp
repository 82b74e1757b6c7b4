// model.hpp -- model parameters, derived step constants and the host-side
// network description of libmc.
//
// The neuron and synapse model is Eq. 1 of Rhodes et al. (arXiv 1909.08665,
// Sec. 2a) integrated exactly over a step; the synaptic store follows Sec. 3a(ii)
// (rows indexed by presynaptic neuron; each synapse = target, weight, delay).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mc {

constexpr int kPops = 8;
constexpr int kPoisMax = 24;          // Poisson CDF thresholds per population
constexpr uint64_t kTagSyn = 1, kTagPois = 2, kTagInit = 3;

enum WeightFormat : int32_t { kWFp32 = 0, kWFp16 = 1, kWBf16 = 2 };

struct ModelParams {
    double conn[64];                  // conn[8*a+b]: pre population a -> post population b
    double full_size[kPops], k_ext[kPops], i_dc[kPops];
    double nu_bg_hz, dt_ms, tau_m_ms, c_m_pf, tau_syn_ms, t_ref_ms, theta_mv;
    double w_mean_pa, w_sd_pa, g, l4e_l23e_factor, w_ext_pa;
    double d_mean_exc_ms, d_sd_exc_ms, d_mean_inh_ms, d_sd_inh_ms;
    double init_u_mean[kPops], init_u_sd[kPops], init_i_mean[kPops], init_i_sd[kPops];   // relaxed start
    int32_t wfmt, poisson_on, init_mode;
};

// Per-step constants of the exact integration, rounded once to float, and the
// Poisson thresholds.  Computed in double on the host.
struct StepConstants {
    float p22, p11, p21, theta;
    float cdc[kPops];                 // P20 * I_dc per population (float)
    int32_t ref_steps;
    int32_t wq_ext;                   // background weight in 1/256 pA
    uint64_t pois_thr[kPops][kPoisMax];
};

// One instance (or a whole batch, with instance-local blocks) in host memory,
// CSR by presynaptic neuron, each row sorted by (target, delay, weight).
struct HostNet {
    int32_t n_inst = 0;
    std::vector<int32_t> inst_off;    // [n_inst+1] first global neuron id of each instance
    std::vector<int64_t> inst_syn_off;// [n_inst+1] first synapse of each instance
    std::vector<uint64_t> seeds;      // [n_inst]
    std::vector<double> scales;       // [n_inst]
    std::vector<int32_t> pop_off;     // [n_inst*(kPops+1)] global population offsets
    std::vector<uint32_t> meta;       // [N] (instance << 3) | population
    int64_t n = 0, m = 0;
    std::vector<uint64_t> row_ptr;    // [N+1]
    std::vector<int32_t> tgt;         // [M] global target id
    std::vector<int32_t> wq;          // [M] weight in 1/256 pA
    std::vector<uint16_t> w16;        // [M] FP16/BF16 bits (reduced-precision stores)
    std::vector<uint8_t> d;           // [M] delay in steps
    std::vector<float> u0;            // [N] initial u
    std::vector<float> i0;            // [N] initial synaptic current
    int32_t ring = 2;                 // power of two > max delay
};

void derive_constants(const ModelParams &p, StepConstants &c);

// The synapses of one (instance, pre population a, post population b) pair:
// global synapse indices [first, first + count), drawn with counter
// (index - first, 8a + b, 0, kTagSyn) and key (seed of the instance, 0).
struct SynSeg {
    int32_t inst, a, b;
    int64_t first, count;
};

// Build one or more instances.  Returns 0 or an MC_ERR_* code with msg set.
int build_host_network(const ModelParams &p, const uint64_t *seeds, const double *scales,
                       int32_t n_inst, HostNet &out, std::string &msg);

// Everything but the synapses: sizes, per-pair counts (as segments), neuron
// metadata and initial state.  H.row_ptr, tgt, wq, w16, d and ring stay empty.
int plan_network(const ModelParams &p, const uint64_t *seeds, const double *scales, int32_t n_inst, HostNet &H,
                 std::vector<SynSeg> &segs, std::string &msg);

// Relaxed initial state (init_mode 2) of instance-local neuron `local` of population a.
void relaxed_start(const ModelParams &p, uint64_t local, int a, uint64_t seed, double &u, double &cur);

// Reduced-precision rounding (round-to-nearest-even from double), as bit patterns.
uint16_t half_bits_rne(double x);
uint16_t bf16_bits_rne(double x);
double half_value(uint16_t h);
double bf16_value(uint16_t h);

}  // namespace mc
