// netbuild.cpp -- host-side construction of the microcircuit synapse store.
//
// Connectivity (Sec. 2a of Rhodes et al., arXiv 1909.08665): populations are
// wired pairwise "based on probability"; here each ordered pair (a -> b) receives
// a fixed total K = log(1-p)/log(1-1/(N_a N_b)) (rounded) of synapses whose pre
// and post are uniform in a and b (with replacement).  Weights are normal
// (87.8 +- 8.78 pA for excitatory sources, mean doubled for L4E -> L2/3E,
// inhibitory = -4 x excitatory), delays normal (workload values), rounded to the
// step and clipped to [1, 255] steps -- the 255-slot input buffer of Sec. 3a(ii).
// Weights crossing zero are clipped at zero (Dale's law, Sec. 2c).
//
// Every random number is one Philox4x64-10 block (Salmon et al., SC'11) with key
// (seed, 0) and counter (synapse index within the pair, 8a+b, 0, 1); the
// per-neuron initial potential uses counter (neuron, 0, 0, 3).
//
// The result is CSR by presynaptic neuron with each row sorted by (target,
// delay, weight) -- the order the tiled engine needs to cut a row into per-tile
// sub-rows with a single pointer per (row, tile).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "model.hpp"
#include "../../include/mc.h"

namespace mc {
namespace {

// ---- Philox4x64-10 on the host ---------------------------------------------
struct Block4 { uint64_t v[4]; };

inline void mul_wide(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    const unsigned __int128 p = static_cast<unsigned __int128>(a) * b;
    hi = static_cast<uint64_t>(p >> 64);
    lo = static_cast<uint64_t>(p);
}

Block4 philox_host(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t seed)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL, kMulB = 0xCA5A826395121157ULL;
    constexpr uint64_t kBumpA = 0x9E3779B97F4A7C15ULL, kBumpB = 0xBB67AE8584CAA73BULL;
    uint64_t key0 = seed, key1 = 0;
    for (int round = 0; round < 10; ++round) {
        uint64_t hA, lA, hB, lB;
        mul_wide(kMulA, c0, hA, lA);
        mul_wide(kMulB, c2, hB, lB);
        const uint64_t x0 = hB ^ c1 ^ key0;
        const uint64_t x2 = hA ^ c3 ^ key1;
        c0 = x0; c1 = lB; c2 = x2; c3 = lA;
        key0 += kBumpA;
        key1 += kBumpB;
    }
    return Block4{{c0, c1, c2, c3}};
}

inline double unit_open_high(uint64_t x) { return std::ldexp(static_cast<double>(x >> 11), -53); }
inline double unit_open_low(uint64_t x) { return std::ldexp(static_cast<double>((x >> 11) + 1), -53); }
inline int64_t scale_to(uint64_t x, int64_t n)
{
    return static_cast<int64_t>((static_cast<unsigned __int128>(x) * static_cast<uint64_t>(n)) >> 64);
}

int thread_count()
{
    int t = static_cast<int>(std::thread::hardware_concurrency());
    if (const char *e = std::getenv("MC_BUILD_THREADS")) t = std::atoi(e);
    return std::max(1, std::min(t, 64));
}

template <class F>
void parallel_ranges(int64_t total, F &&fn)
{
    const int nt = thread_count();
    if (nt == 1 || total < 4096) { fn(int64_t{0}, total); return; }
    std::vector<std::thread> pool;
    const int64_t chunk = (total + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int64_t a = t * chunk, b = std::min(total, a + chunk);
        if (a >= b) break;
        pool.emplace_back([&fn, a, b] { fn(a, b); });
    }
    for (auto &th : pool) th.join();
}

struct Syn {
    int32_t tgt;
    int32_t wq;
    uint16_t w16;
    uint8_t d;
};

bool syn_less(const Syn &x, const Syn &y)
{
    if (x.tgt != y.tgt) return x.tgt < y.tgt;
    if (x.d != y.d) return x.d < y.d;
    return x.wq < y.wq;
}

}  // namespace

// ---- reduced-precision rounding -------------------------------------------------
// Round-to-nearest-even straight from double to the bit pattern of a binary
// floating-point format with `frac` stored fraction bits and exponent bias `bias`.
static uint16_t rne_bits(double x, int frac, int bias, int max_exp_field)
{
    const uint16_t sign = std::signbit(x) ? static_cast<uint16_t>(1u << (frac + (max_exp_field == 31 ? 5 : 8))) : 0;
    const double a = std::fabs(x);
    if (a == 0.0) return sign;
    int e = std::ilogb(a);                    // a in [2^e, 2^(e+1))
    const int emin = 1 - bias;
    if (e < emin) {                           // subnormal: units of 2^(emin-frac)
        const double m = std::nearbyint(std::ldexp(a, frac - emin));
        return static_cast<uint16_t>(sign | static_cast<uint16_t>(m));   // m == 2^frac -> smallest normal
    }
    double m = std::nearbyint(std::ldexp(a, frac - e));                // in [2^frac, 2^(frac+1)]
    if (m == std::ldexp(1.0, frac + 1)) { m = std::ldexp(1.0, frac); e += 1; }
    const int field = e + bias;
    if (field >= max_exp_field) return static_cast<uint16_t>(sign | (max_exp_field << frac));   // infinity
    return static_cast<uint16_t>(sign | (field << frac) | (static_cast<int>(m) - (1 << frac)));
}

uint16_t half_bits_rne(double x) { return rne_bits(x, 10, 15, 31); }
uint16_t bf16_bits_rne(double x) { return rne_bits(x, 7, 127, 255); }

double half_value(uint16_t h)
{
    const int s = h >> 15, f = (h >> 10) & 31, m = h & 1023;
    double v = f == 0 ? std::ldexp(m, -24) : std::ldexp(1024 + m, f - 25);
    if (f == 31) v = m ? NAN : INFINITY;
    return s ? -v : v;
}

double bf16_value(uint16_t h)
{
    const uint32_t bits = static_cast<uint32_t>(h) << 16;
    float f;
    std::memcpy(&f, &bits, 4);
    return f;
}

// ---- step constants ---------------------------------------------------------
void derive_constants(const ModelParams &p, StepConstants &c)
{
    // Exact integration of Eq. 1 over one step dt (linear system in u = V - E_L
    // and I): u' = P22 u + P21 I + P20 I_dc, I' = P11 I + input.
    const double p22 = std::exp(-p.dt_ms / p.tau_m_ms);
    const double p11 = std::exp(-p.dt_ms / p.tau_syn_ms);
    const double p21 = ((p.tau_m_ms * p.tau_syn_ms) / (p.c_m_pf * (p.tau_m_ms - p.tau_syn_ms))) * (p22 - p11);
    const double p20 = (p.tau_m_ms / p.c_m_pf) * (1.0 - p22);
    c.p22 = static_cast<float>(p22);
    c.p11 = static_cast<float>(p11);
    c.p21 = static_cast<float>(p21);
    c.theta = static_cast<float>(p.theta_mv);
    for (int a = 0; a < kPops; ++a) c.cdc[a] = static_cast<float>(p20 * p.i_dc[a]);
    c.ref_steps = static_cast<int32_t>(std::llround(p.t_ref_ms / p.dt_ms));

    double wext = p.w_ext_pa;
    if (p.wfmt == kWFp16) wext = half_value(half_bits_rne(wext));
    else if (p.wfmt == kWBf16) wext = bf16_value(bf16_bits_rne(wext));
    c.wq_ext = static_cast<int32_t>(std::nearbyint(wext * 256.0));

    // Poisson count by inversion: thresholds floor(2^32 * CDF(k)), k < kPoisMax,
    // rate 8 Hz * K_ext per neuron (Sec. 3a(iii)).
    for (int a = 0; a < kPops; ++a) {
        const double lambda = ((p.nu_bg_hz * p.k_ext[a]) * p.dt_ms) * 1e-3;
        double term = std::exp(-lambda);
        double cdf = term;
        for (int k = 0; k < kPoisMax; ++k) {
            if (k) {
                term = (term * lambda) / static_cast<double>(k);
                cdf = cdf + term;
            }
            c.pois_thr[a][k] = cdf >= 1.0 ? (uint64_t{1} << 32) : static_cast<uint64_t>(std::floor(cdf * 4294967296.0));
        }
    }
}

// Relaxed initial state of neuron `local` of population a (init_mode 2; the
// paper starts from potentials that make the first steps look like the steady
// state, Sec. 4a).  Block (local, 1 + r, 0, kTagInit) gives a normal pair by
// Box-Muller on words 0 and 1 and a uniform in word 2.  The synaptic current
// is i_mean + i_sd * (second normal of the first block).  The potential is
// u_mean + u_sd * (first normal) of the first block r whose value lies below
// theta and whose uniform passes 1 - exp(-2 (theta - u)(theta - u_mean) / u_sd^2):
// the normal density minus its mirror image in the threshold, which vanishes
// at theta as the steady state's does.
void relaxed_start(const ModelParams &p, uint64_t local, int a, uint64_t seed, double &u, double &cur)
{
    const double mu = p.init_u_mean[a], sd = p.init_u_sd[a], th = p.theta_mv;
    const double two_pi = 6.283185307179586;
    u = 0.0;
    cur = 0.0;
    for (uint64_t r = 0; r < 64; ++r) {
        const Block4 x = philox_host(local, 1 + r, 0, kTagInit, seed);
        const double radius = std::sqrt(-2.0 * std::log(unit_open_low(x.v[0])));
        const double angle = two_pi * unit_open_high(x.v[1]);
        const double z1 = radius * std::cos(angle);
        if (r == 0) cur = p.init_i_mean[a] + p.init_i_sd[a] * (radius * std::sin(angle));
        const double v = mu + sd * z1;
        const double accept = 1.0 - std::exp(-2.0 * (th - v) * (th - mu) / (sd * sd));
        if (v < th && unit_open_high(x.v[2]) < accept) {
            u = v;
            return;
        }
    }
}

// ---- network ------------------------------------------------------------------
int plan_network(const ModelParams &p, const uint64_t *seeds, const double *scales, int32_t n_inst, HostNet &out,
                 std::vector<SynSeg> &segs, std::string &msg)
{
    if (n_inst < 1) { msg = "at least one instance is required"; return MC_ERR_ARG; }
    for (int q = 0; q < 64; ++q)
        if (!(p.conn[q] >= 0.0 && p.conn[q] < 1.0)) { msg = "connection probabilities must lie in [0, 1)"; return MC_ERR_ARG; }

    HostNet &H = out;
    H.n_inst = n_inst;
    H.inst_off.assign(n_inst + 1, 0);
    H.inst_syn_off.assign(n_inst + 1, 0);
    H.seeds.assign(seeds, seeds + n_inst);
    H.scales.assign(scales, scales + n_inst);
    H.pop_off.assign(static_cast<size_t>(n_inst) * (kPops + 1), 0);

    // Sizes and per-pair synapse counts of every instance.
    std::vector<int64_t> pair_k(static_cast<size_t>(n_inst) * 64);
    int64_t n_total = 0, m_total = 0;
    for (int j = 0; j < n_inst; ++j) {
        const double s = scales[j];
        if (!(s > 0.0 && s <= 1.0)) { msg = "scale must be in (0, 1]"; return MC_ERR_ARG; }
        int32_t *po = &H.pop_off[static_cast<size_t>(j) * (kPops + 1)];
        po[0] = static_cast<int32_t>(n_total);
        int64_t sz[kPops];
        for (int a = 0; a < kPops; ++a) {
            sz[a] = std::max<int64_t>(1, static_cast<int64_t>(std::floor(p.full_size[a] * s + 0.5)));
            po[a + 1] = po[a] + static_cast<int32_t>(sz[a]);
        }
        H.inst_off[j] = static_cast<int32_t>(n_total);
        H.inst_syn_off[j] = m_total;
        for (int a = 0; a < kPops; ++a)
            for (int b = 0; b < kPops; ++b) {
                const double pr = p.conn[8 * a + b];
                int64_t k = 0;
                if (pr > 0.0) {
                    const double pairs = static_cast<double>(sz[a]) * static_cast<double>(sz[b]);
                    k = std::llround(std::log1p(-pr) / std::log1p(-1.0 / pairs));
                }
                pair_k[static_cast<size_t>(j) * 64 + 8 * a + b] = k;
                m_total += k;
            }
        n_total = po[kPops];
        if (n_total >= (int64_t{1} << 31)) { msg = "too many neurons"; return MC_ERR_ARG; }
    }
    H.inst_off[n_inst] = static_cast<int32_t>(n_total);
    H.inst_syn_off[n_inst] = m_total;
    H.n = n_total;
    H.m = m_total;

    H.meta.resize(n_total);
    for (int j = 0; j < n_inst; ++j) {
        const int32_t *po = &H.pop_off[static_cast<size_t>(j) * (kPops + 1)];
        for (int a = 0; a < kPops; ++a)
            for (int32_t i = po[a]; i < po[a + 1]; ++i) H.meta[i] = (static_cast<uint32_t>(j) << 3) | static_cast<uint32_t>(a);
    }

    // Enumerate (instance, pair) segments of the global synapse index space.
    segs.clear();
    {
        int64_t at = 0;
        for (int j = 0; j < n_inst; ++j)
            for (int q = 0; q < 64; ++q) {
                const int64_t k = pair_k[static_cast<size_t>(j) * 64 + q];
                if (k) segs.push_back(SynSeg{j, q / 8, q % 8, at, k});
                at += k;
            }
    }

    // Initial state: u ~ U[0, theta) (init_mode 0), all zero (1), or the relaxed
    // start (2).
    H.u0.assign(n_total, 0.0f);
    H.i0.assign(n_total, 0.0f);
    if (p.init_mode == 0) {
        for (int j = 0; j < n_inst; ++j)
            for (int32_t i = H.inst_off[j]; i < H.inst_off[j + 1]; ++i) {
                const Block4 x = philox_host(static_cast<uint64_t>(i - H.inst_off[j]), 0, 0, kTagInit, H.seeds[j]);
                H.u0[i] = static_cast<float>(p.theta_mv * unit_open_high(x.v[0]));
            }
    } else if (p.init_mode == 2) {
        for (int j = 0; j < n_inst; ++j)
            for (int32_t i = H.inst_off[j]; i < H.inst_off[j + 1]; ++i) {
                double u = 0.0, cur = 0.0;
                relaxed_start(p, static_cast<uint64_t>(i - H.inst_off[j]), static_cast<int>(H.meta[i] & 7u), H.seeds[j], u, cur);
                H.u0[i] = static_cast<float>(u);
                H.i0[i] = static_cast<float>(cur);
            }
    }
    return MC_OK;
}

int build_host_network(const ModelParams &p, const uint64_t *seeds, const double *scales, int32_t n_inst,
                       HostNet &out, std::string &msg)
{
    std::vector<SynSeg> segs;
    int rc = plan_network(p, seeds, scales, n_inst, out, segs, msg);
    if (rc) return rc;
    HostNet &H = out;
    const int64_t n_total = H.n, m_total = H.m;
    auto seg_of = [&segs](int64_t s) {
        size_t lo = 0, hi = segs.size();
        while (hi - lo > 1) {
            const size_t mid = (lo + hi) / 2;
            if (segs[mid].first <= s) lo = mid; else hi = mid;
        }
        return lo;
    };

    auto pre_of = [&](const SynSeg &sg, const Block4 &x) {
        const int32_t *po = &H.pop_off[static_cast<size_t>(sg.inst) * (kPops + 1)];
        return po[sg.a] + static_cast<int32_t>(scale_to(x.v[0], po[sg.a + 1] - po[sg.a]));
    };

    // Pass 1: out-degree of every neuron (only the pre draw is needed).
    std::vector<std::atomic<uint64_t>> fill(static_cast<size_t>(n_total) + 1);
    for (auto &f : fill) f.store(0, std::memory_order_relaxed);
    parallel_ranges(m_total, [&](int64_t s0, int64_t s1) {
        if (s0 >= s1) return;
        size_t g = seg_of(s0);
        for (int64_t s = s0; s < s1; ++s) {
            while (s >= segs[g].first + segs[g].count) ++g;
            const SynSeg &sg = segs[g];
            const Block4 x = philox_host(static_cast<uint64_t>(s - sg.first), static_cast<uint64_t>(8 * sg.a + sg.b), 0,
                                         kTagSyn, H.seeds[sg.inst]);
            fill[pre_of(sg, x) + 1].fetch_add(1, std::memory_order_relaxed);
        }
    });
    H.row_ptr.assign(static_cast<size_t>(n_total) + 1, 0);
    for (int64_t i = 0; i < n_total; ++i) H.row_ptr[i + 1] = H.row_ptr[i] + fill[i + 1].load();
    for (int64_t i = 0; i < n_total; ++i) fill[i].store(H.row_ptr[i], std::memory_order_relaxed);

    // Pass 2: full draw of every synapse, scattered into its row.
    std::vector<Syn> syn;
    try { syn.resize(static_cast<size_t>(m_total)); } catch (...) { msg = "out of host memory"; return MC_ERR_NOMEM; }
    std::atomic<int> bad{0};
    const double two_pi = 6.283185307179586;
    parallel_ranges(m_total, [&](int64_t s0, int64_t s1) {
        if (s0 >= s1) return;
        size_t g = seg_of(s0);
        for (int64_t s = s0; s < s1; ++s) {
            while (s >= segs[g].first + segs[g].count) ++g;
            const SynSeg &sg = segs[g];
            const int32_t *po = &H.pop_off[static_cast<size_t>(sg.inst) * (kPops + 1)];
            const Block4 x = philox_host(static_cast<uint64_t>(s - sg.first), static_cast<uint64_t>(8 * sg.a + sg.b), 0,
                                         kTagSyn, H.seeds[sg.inst]);
            const int32_t pre = pre_of(sg, x);
            const int32_t post = po[sg.b] + static_cast<int32_t>(scale_to(x.v[1], po[sg.b + 1] - po[sg.b]));
            // Box-Muller pair: one normal for the weight, one for the delay.
            const double radius = std::sqrt(-2.0 * std::log(unit_open_low(x.v[2])));
            const double angle = two_pi * unit_open_high(x.v[3]);
            const double z_w = radius * std::cos(angle);
            const double z_d = radius * std::sin(angle);
            const bool excitatory = (sg.a % 2) == 0;
            double mean = excitatory ? p.w_mean_pa : p.g * p.w_mean_pa;
            const double sd = excitatory ? p.w_sd_pa : std::fabs(p.g) * p.w_sd_pa;
            if (sg.a == 2 && sg.b == 0) mean = p.l4e_l23e_factor * p.w_mean_pa;
            double w = mean + sd * z_w;
            if (excitatory) w = std::max(w, 0.0); else w = std::min(w, 0.0);
            const double dmean = excitatory ? p.d_mean_exc_ms : p.d_mean_inh_ms;
            const double dsd = excitatory ? p.d_sd_exc_ms : p.d_sd_inh_ms;
            double dsteps = std::nearbyint((dmean + dsd * z_d) / p.dt_ms);
            dsteps = std::min(255.0, std::max(1.0, dsteps));

            Syn e;
            e.tgt = post;
            e.d = static_cast<uint8_t>(dsteps);
            e.w16 = 0;
            double stored = w;
            if (p.wfmt == kWFp16) { e.w16 = half_bits_rne(w); stored = half_value(e.w16); }
            else if (p.wfmt == kWBf16) { e.w16 = bf16_bits_rne(w); stored = bf16_value(e.w16); }
            const double q = std::nearbyint(stored * 256.0);
            if (!(std::fabs(q) < 16777216.0)) bad.store(1);
            e.wq = static_cast<int32_t>(q);
            syn[fill[pre].fetch_add(1, std::memory_order_relaxed)] = e;
        }
    });
    fill.clear();
    fill.shrink_to_fit();
    if (bad.load()) { msg = "a weight exceeds the 2^24/256 pA range of the fixed-point store"; return MC_ERR_ARG; }

    // Canonical row order.
    parallel_ranges(n_total, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            std::sort(syn.begin() + static_cast<int64_t>(H.row_ptr[i]), syn.begin() + static_cast<int64_t>(H.row_ptr[i + 1]), syn_less);
    });

    // Structure-of-arrays store, ring depth and the int32 accumulation bound.
    try {
        H.tgt.resize(m_total);
        H.wq.resize(m_total);
        H.d.resize(m_total);
        if (p.wfmt != kWFp32) H.w16.resize(m_total);
    } catch (...) { msg = "out of host memory"; return MC_ERR_NOMEM; }
    std::atomic<int> maxd{1};
    parallel_ranges(m_total, [&](int64_t s0, int64_t s1) {
        int md = 1;
        for (int64_t s = s0; s < s1; ++s) {
            H.tgt[s] = syn[s].tgt;
            H.wq[s] = syn[s].wq;
            H.d[s] = syn[s].d;
            if (!H.w16.empty()) H.w16[s] = syn[s].w16;
            md = std::max<int>(md, syn[s].d);
        }
        int cur = maxd.load();
        while (md > cur && !maxd.compare_exchange_weak(cur, md)) {}
    });
    std::vector<Syn>().swap(syn);
    int ring = 2;
    while (ring < maxd.load() + 1) ring *= 2;
    H.ring = ring;

    StepConstants sc;
    derive_constants(p, sc);
    {
        std::vector<int64_t> in_abs(static_cast<size_t>(n_total), 0);
        for (int64_t s = 0; s < m_total; ++s) in_abs[H.tgt[s]] += std::llabs(static_cast<long long>(H.wq[s]));
        const int64_t pois_max = static_cast<int64_t>(kPoisMax) * std::llabs(static_cast<long long>(sc.wq_ext));
        for (int64_t i = 0; i < n_total; ++i)
            if (in_abs[i] + pois_max >= (int64_t{1} << 31)) {
                msg = "int32 input-buffer overflow bound exceeded";
                return MC_ERR_OVERFLOW_BOUND;
            }
    }
    return MC_OK;
}

}  // namespace mc
