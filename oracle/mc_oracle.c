/*
 * mc_oracle.c -- CPU oracle for the fixed-step cortical-microcircuit simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  The simulator (the HIP library)
 * never links, loads or calls it, and this file shares no code with it.
 *
 * It is the plain, slow, obviously-correct statement of what one simulation step
 * computes, following Rhodes et al., "Real-Time Cortical Simulation on
 * Neuromorphic Hardware" (arXiv 1909.08665):
 *
 *   - the neuron model: Sec. 2a, Eq. 1 -- leaky integrate-and-fire membrane with a
 *     current-based, exponentially decaying synaptic current; a spike is emitted
 *     when V exceeds the threshold and V is set to the reset potential;
 *   - weights and delays: Sec. 2a -- normal weights (87.8 +- 8.78 pA for excitatory
 *     sources, doubled mean for layer-4 -> layer-2/3 excitatory, inhibitory scaled
 *     by -4), normal delays rounded to the time step;
 *   - synaptic rows indexed by the presynaptic neuron, each synapse adding its
 *     weight into the target's input-buffer slot `delay` steps ahead, and the slot
 *     for the current step being consumed and cleared: Sec. 3a(ii);
 *   - Poisson background: each step, how many background spikes arrive, times the
 *     background weight, added to the step's synaptic input: Sec. 3a(ii), with the
 *     8 Hz x K_ext source rates of Sec. 3a(iii);
 *   - a synaptic event is one spike reaching one postsynaptic synapse: Sec. 3c.
 *
 * Points the paper leaves open are fixed as follows (each is a stated reading):
 *   R1 Eq. 1 is printed with garbled signs; the leaky forms -(V-E) and -I/tau_syn
 *      are used (the text says the current decays).
 *   R2 Threshold test is strict (V > V_theta), V is then held at V_reset for the
 *      refractory time t_ref = 2 ms (20 steps) while I keeps integrating.
 *   R3 Exact integration of the linear system over one step:
 *         u <- P22*u + P21*I   (+ P20*I_dc)      using I from the previous step,
 *         I <- P11*I + input(step)
 *      so input arriving at step n moves V from step n+1 on.  u = V - E_L.
 *   R4 Connectivity: fixed total number K_ab per ordered population pair,
 *      K = log(1-p)/log(1-1/(N_pre*N_post)) rounded to nearest, with pre and post
 *      drawn uniformly with replacement (multapses and autapses allowed).
 *   R5 Delays: rint(delay/dt), clipped to [1, 255] steps (255 = buffer slots).
 *   R6 Weights that cross zero are clipped at zero, keeping Dale's law.
 *   R7 Background weight is 87.8 pA, fixed; background spikes enter I in the step
 *      they are drawn.  Count ~ Poisson(8 Hz * K_ext * dt) by integer inversion of
 *      a 32-bit uniform against K_MAX fixed-point CDF thresholds.
 *   R8 Initial state: u ~ U[0, theta), I = 0, not refractory (init_mode 0), or all zero
 *      (1), or a relaxed start (2; Sec. 4a: initial potentials chosen so that the
 *      first steps look like the steady state, values not given): per population
 *      I ~ N(mu_I, sd_I) and u drawn from the density of N(mu_u, sd_u) with an
 *      absorbing threshold, phi((u-mu)/sd) - phi((u-(2 theta-mu))/sd) for u < theta
 *      (the method of images), by rejection; the moments are inputs.
 *   R9 Random numbers: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 *      counter (c0, c1, c2, tag) -- one block per synapse and per neuron initial
 *      value; one block per step and group of 8 consecutive neurons for the
 *      Poisson draws, neuron i taking 32-bit half (i mod 8) of the 256 bits
 *      (halves ordered high, low of word 0, then of words 1, 2, 3).
 *   R10 FP32 mirror: every product and sum rounded to float, no fused multiply-add;
 *      synaptic input accumulated as int32 in units of 1/256 pA (Q8), converted to
 *      float with round-to-nearest-even and scaled by 2^-8 (exact).
 *      FP64 mode: double state, unquantised weights, double input buffer.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#pragma STDC FP_CONTRACT OFF

#define OR_NPOP 8
#define OR_KMAX 24
#define TAG_SYN 1u
#define TAG_POIS 2u
#define TAG_INIT 3u

/* ------------------------------------------------------------------------- */
/* Error reporting                                                           */
/* ------------------------------------------------------------------------- */
static char g_err[512];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *or_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64   */
/* multiplies with a Weyl-sequence key schedule.                              */
/* ------------------------------------------------------------------------- */
void or_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u53(uint64_t x) { return (double)(x >> 11) * 0x1p-53; }          /* [0,1) */
static double u53p(uint64_t x) { return (double)((x >> 11) + 1) * 0x1p-53; }   /* (0,1] */
static int64_t mulhi_n(uint64_t x, int64_t n)                                  /* floor(x*n/2^64) */
{
    return (int64_t)(((unsigned __int128)x * (uint64_t)n) >> 64);
}

/* ------------------------------------------------------------------------- */
/* Round-to-nearest-even of a double to binary16 / bfloat16, returned as a     */
/* double holding the exactly representable value.                            */
/* ------------------------------------------------------------------------- */
static double round_to_format(double x, int mant_bits, int emin)
{
    /* mant_bits: stored fraction bits (10 for binary16, 7 for bfloat16);
       emin: exponent of the smallest normal number. */
    if (x == 0.0 || !isfinite(x)) return x;
    double a = fabs(x);
    int ex;
    frexp(a, &ex);                 /* a = m * 2^ex, m in [0.5, 1) */
    int e = ex - 1;                /* a in [2^e, 2^(e+1)) */
    if (e < emin) e = emin;        /* subnormal range keeps the smallest quantum */
    double q = ldexp(1.0, e - mant_bits);
    double r = rint(a / q) * q;    /* a/q is exact: q is a power of two */
    return x < 0 ? -r : r;
}
double or_round_fp16(double x) { return round_to_format(x, 10, -14); }
double or_round_bf16(double x) { return round_to_format(x, 7, -126); }

/* ------------------------------------------------------------------------- */
/* Parameters and network                                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t mode;            /* 0 = FP32 mirror, 1 = FP64 */
    int32_t wfmt;            /* weight store in mirror mode: 0 FP32(Q8), 1 FP16, 2 BF16 */
    int32_t poisson_on;      /* 1 = Poisson background drive */
    int32_t init_mode;       /* 0 = u ~ U[0,theta), 1 = all zero */
    double full_size[OR_NPOP];
    double k_ext[OR_NPOP];
    double i_dc_pa[OR_NPOP];
    double nu_bg_hz, dt_ms;
    double tau_m_ms, c_m_pf, tau_syn_ms, t_ref_ms, theta_mv;
    double w_mean_pa, w_sd_pa, g, l4e_l23e_factor, w_ext_pa;
    double d_mean_exc_ms, d_sd_exc_ms, d_mean_inh_ms, d_sd_inh_ms;
    uint64_t pois_stream;    /* second key word of the Poisson draws: 0 for the model; other
                                values give independent background realisations on the same
                                network (noise-floor estimates only) */
    double init_u_mean_mv[OR_NPOP], init_u_sd_mv[OR_NPOP];   /* relaxed start (init_mode 2) */
    double init_i_mean_pa[OR_NPOP], init_i_sd_pa[OR_NPOP];
} or_params;

typedef struct {
    or_params p;
    uint64_t seed;
    int32_t N, R, ref_steps;
    int32_t pop_size[OR_NPOP], pop_off[OR_NPOP + 1];
    int64_t M;
    int64_t *row_ptr;
    int32_t *post, *wq;
    double *w64;
    uint8_t *d;
    /* constants */
    double P22, P11, P21, P20, theta, w_ext;
    float P22f, P11f, P21f, thetaf, cdc_f[OR_NPOP];
    double cdc_d[OR_NPOP];
    int32_t wq_ext;
    uint64_t T[OR_NPOP][OR_KMAX];
    /* state */
    int64_t step;
    float *uf, *If;
    double *ud, *Id;
    int32_t *refr;
    int32_t *ring;
    double *ringd;
    uint8_t *spk;       /* per-neuron spike flag of the current step */
    int32_t *pop_of;
    /* spike record */
    int64_t nrec, caprec;
    int64_t *rec_step;
    int32_t *rec_id;
    /* counters */
    int64_t n_spikes, n_events, n_pois;
    int32_t max_s;
} or_net;

static int is_exc(int pop) { return (pop % 2) == 0; }   /* L2/3E, L2/3I, L4E, ... */

void or_free(or_net *nt)
{
    if (!nt) return;
    free(nt->row_ptr); free(nt->post); free(nt->wq); free(nt->w64); free(nt->d);
    free(nt->uf); free(nt->If); free(nt->ud); free(nt->Id); free(nt->refr);
    free(nt->ring); free(nt->ringd); free(nt->spk); free(nt->pop_of);
    free(nt->rec_step); free(nt->rec_id);
    free(nt);
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Integer weight in units of 1/256 pA for the mirror modes (reading R10). */
static int quantise(const or_params *p, double w, int32_t *out)
{
    double v = w;
    if (p->wfmt == 1) v = or_round_fp16(w);
    else if (p->wfmt == 2) v = or_round_bf16(w);
    double s = rint(v * 256.0);
    if (!(fabs(s) < 2147483648.0)) return -1;
    *out = (int32_t)s;
    return 0;
}

/* Constants of the exact integration over one step (reading R3), computed in
   double and rounded once to float for the mirror. */
static void compute_constants(or_net *nt)
{
    const or_params *p = &nt->p;
    nt->P22 = exp(-p->dt_ms / p->tau_m_ms);
    nt->P11 = exp(-p->dt_ms / p->tau_syn_ms);
    nt->P21 = ((p->tau_m_ms * p->tau_syn_ms) / (p->c_m_pf * (p->tau_m_ms - p->tau_syn_ms))) * (nt->P22 - nt->P11);
    nt->P20 = (p->tau_m_ms / p->c_m_pf) * (1.0 - nt->P22);
    nt->theta = p->theta_mv;
    nt->P22f = (float)nt->P22;
    nt->P11f = (float)nt->P11;
    nt->P21f = (float)nt->P21;
    nt->thetaf = (float)nt->theta;
    nt->ref_steps = (int32_t)llround(p->t_ref_ms / p->dt_ms);
    for (int a = 0; a < OR_NPOP; ++a) {
        nt->cdc_d[a] = nt->P20 * p->i_dc_pa[a];
        nt->cdc_f[a] = (float)nt->cdc_d[a];
    }
    /* Poisson CDF thresholds (reading R7): lambda = 8 Hz * K_ext * dt. */
    for (int a = 0; a < OR_NPOP; ++a) {
        double lam = ((p->nu_bg_hz * p->k_ext[a]) * p->dt_ms) * 1e-3;
        double pk = exp(-lam), F = pk;
        for (int k = 0; k < OR_KMAX; ++k) {
            if (k > 0) {
                pk = (pk * lam) / (double)k;
                F = F + pk;
            }
            nt->T[a][k] = (F >= 1.0) ? (1ULL << 32) : (uint64_t)floor(ldexp(F, 32));
        }
    }
}

/* Relaxed initial state of neuron i (instance-local index) of population a
   (reading R8, init_mode 2).  Block (i, 1 + r, 0, TAG_INIT) gives the normal
   pair (z1, z2) by Box-Muller on its words 0 and 1 and a uniform in word 2:
   I takes mu_I + sd_I z2 of the first block; u takes mu_u + sd_u z1 of the first
   block r whose value lies below theta and whose uniform is below the image
   density's acceptance ratio 1 - exp(-2 (theta - u)(theta - mu_u) / sd_u^2). */
static void relaxed_state(const or_net *nt, int32_t i, int a, double *u, double *I)
{
    const double mu = nt->p.init_u_mean_mv[a], sd = nt->p.init_u_sd_mv[a], th = nt->theta;
    const double two_pi = 6.283185307179586;
    *u = 0.0;
    for (int r = 0; r < 64; ++r) {
        uint64_t c[4] = {(uint64_t)i, (uint64_t)(1 + r), 0, TAG_INIT}, k[2] = {nt->seed, 0}, x[4];
        or_philox(c, k, x);
        const double rad = sqrt(-2.0 * log(u53p(x[0])));
        const double phi = two_pi * u53(x[1]);
        const double z1 = rad * cos(phi);
        if (r == 0) *I = nt->p.init_i_mean_pa[a] + nt->p.init_i_sd_pa[a] * (rad * sin(phi));
        const double v = mu + sd * z1;
        const double accept = 1.0 - exp(-2.0 * (th - v) * (th - mu) / (sd * sd));
        if (v < th && u53(x[2]) < accept) {
            *u = v;
            return;
        }
    }
}

/* Counting sort of the synapse list by presynaptic neuron (stable), then the
   ring depth, the int32 bound and the initial state. */
static int finish_network(or_net *nt, int32_t *pre, int32_t *post, int32_t *wq,
                          double *w64, uint8_t *d)
{
    const int32_t N = nt->N;
    const int64_t M = nt->M;
    nt->row_ptr = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    nt->post = (int32_t *)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
    nt->wq = (int32_t *)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
    nt->d = (uint8_t *)malloc((size_t)(M ? M : 1));
    if (w64) nt->w64 = (double *)malloc((size_t)(M ? M : 1) * sizeof(double));
    if (!nt->row_ptr || !nt->post || !nt->wq || !nt->d || (w64 && !nt->w64)) {
        set_err("out of host memory");
        return -1;
    }
    for (int64_t s = 0; s < M; ++s) nt->row_ptr[pre[s] + 1]++;
    for (int32_t i = 0; i < N; ++i) nt->row_ptr[i + 1] += nt->row_ptr[i];
    int64_t *fill = (int64_t *)malloc((size_t)(N ? N : 1) * sizeof(int64_t));
    if (!fill) { set_err("out of host memory"); return -1; }
    memcpy(fill, nt->row_ptr, (size_t)N * sizeof(int64_t));
    int maxd = 0;
    for (int64_t s = 0; s < M; ++s) {
        int64_t at = fill[pre[s]]++;
        nt->post[at] = post[s];
        nt->wq[at] = wq[s];
        nt->d[at] = d[s];
        if (w64) nt->w64[at] = w64[s];
        if (d[s] > maxd) maxd = d[s];
    }
    free(fill);

    /* Ring depth: smallest power of two > max delay, at least 2. */
    int R = 2;
    while (R < maxd + 1) R *= 2;
    nt->R = R;

    compute_constants(nt);
    if (quantise(&nt->p, nt->p.w_ext_pa, &nt->wq_ext) != 0) { set_err("background weight out of range"); return -1; }
    nt->w_ext = nt->p.w_ext_pa;

    /* int32 accumulation bound: every incoming |wq| plus the largest Poisson
       contribution must stay below 2^31 for each neuron. */
    if (nt->p.mode == 0) {
        int64_t *acc = (int64_t *)calloc((size_t)(N ? N : 1), sizeof(int64_t));
        if (!acc) { set_err("out of host memory"); return -1; }
        for (int64_t s = 0; s < M; ++s) acc[nt->post[s]] += llabs((long long)nt->wq[s]);
        int64_t pk = (int64_t)OR_KMAX * llabs((long long)nt->wq_ext);
        for (int32_t i = 0; i < N; ++i) {
            if (acc[i] + pk >= 2147483648LL) { free(acc); set_err("int32 input-buffer overflow bound exceeded"); return -2; }
        }
        free(acc);
    }

    /* State (reading R8). */
    nt->pop_of = (int32_t *)malloc((size_t)(N ? N : 1) * sizeof(int32_t));
    nt->refr = (int32_t *)calloc((size_t)(N ? N : 1), sizeof(int32_t));
    nt->spk = (uint8_t *)calloc((size_t)(N ? N : 1), 1);
    if (!nt->pop_of || !nt->refr || !nt->spk) { set_err("out of host memory"); return -1; }
    for (int a = 0; a < OR_NPOP; ++a)
        for (int32_t i = nt->pop_off[a]; i < nt->pop_off[a + 1]; ++i) nt->pop_of[i] = a;
    if (nt->p.mode == 0) {
        nt->uf = (float *)calloc((size_t)(N ? N : 1), sizeof(float));
        nt->If = (float *)calloc((size_t)(N ? N : 1), sizeof(float));
        nt->ring = (int32_t *)calloc((size_t)R * (size_t)(N ? N : 1), sizeof(int32_t));
        if (!nt->uf || !nt->If || !nt->ring) { set_err("out of host memory"); return -1; }
    } else {
        nt->ud = (double *)calloc((size_t)(N ? N : 1), sizeof(double));
        nt->Id = (double *)calloc((size_t)(N ? N : 1), sizeof(double));
        nt->ringd = (double *)calloc((size_t)R * (size_t)(N ? N : 1), sizeof(double));
        if (!nt->ud || !nt->Id || !nt->ringd) { set_err("out of host memory"); return -1; }
    }
    for (int32_t i = 0; i < N; ++i) {
        double u0 = 0.0, i0 = 0.0;
        if (nt->p.init_mode == 0) {
            uint64_t c[4] = {(uint64_t)i, 0, 0, TAG_INIT}, k[2] = {nt->seed, 0}, x[4];
            or_philox(c, k, x);
            u0 = nt->theta * u53(x[0]);
        } else if (nt->p.init_mode == 2) {
            relaxed_state(nt, i, nt->pop_of[i], &u0, &i0);
        }
        if (nt->p.mode == 0) {
            nt->uf[i] = (float)u0;
            nt->If[i] = (float)i0;
        } else {
            nt->ud[i] = u0;
            nt->Id[i] = i0;
        }
    }
    return 0;
}

static or_net *new_net(const or_params *p, uint64_t seed)
{
    or_net *nt = (or_net *)calloc(1, sizeof(or_net));
    if (!nt) { set_err("out of host memory"); return NULL; }
    nt->p = *p;
    nt->seed = seed;
    return nt;
}

static int check_params(const or_params *p)
{
    if (p->mode != 0 && p->mode != 1) { set_err("mode must be 0 or 1"); return -1; }
    if (p->wfmt < 0 || p->wfmt > 2) { set_err("wfmt must be 0, 1 or 2"); return -1; }
    if (!(p->dt_ms > 0) || !(p->tau_m_ms > 0) || !(p->tau_syn_ms > 0) || !(p->c_m_pf > 0)) {
        set_err("time constants, capacitance and dt must be positive"); return -1;
    }
    if (p->tau_m_ms == p->tau_syn_ms) { set_err("tau_m must differ from tau_syn"); return -1; }
    if (p->init_mode < 0 || p->init_mode > 2) { set_err("init_mode must be 0, 1 or 2"); return -1; }
    if (p->init_mode == 2)
        for (int a = 0; a < OR_NPOP; ++a)
            if (!(p->init_u_sd_mv[a] > 0.0) || !(p->init_u_mean_mv[a] < p->theta_mv) || !(p->init_i_sd_pa[a] >= 0.0)) {
                set_err("relaxed start needs sd_u > 0, mean_u < theta and sd_I >= 0 for every population");
                return -1;
            }
    return 0;
}

/*
 * Build the microcircuit at `scale` from the connection table conn[8*a + b] =
 * probability that a given (pre in population a, post in population b) pair is
 * connected (readings R4-R6, R9).
 */
or_net *or_build(const or_params *p, uint64_t seed, double scale, const double *conn)
{
    if (check_params(p)) return NULL;
    if (!(scale > 0.0) || scale > 1.0) { set_err("scale must be in (0, 1]"); return NULL; }
    for (int q = 0; q < 64; ++q)
        if (!(conn[q] >= 0.0) || !(conn[q] < 1.0)) { set_err("connection probabilities must lie in [0, 1)"); return NULL; }
    or_net *nt = new_net(p, seed);
    if (!nt) return NULL;

    /* Population sizes: floor(N_full * scale + 0.5), at least one neuron. */
    nt->pop_off[0] = 0;
    for (int a = 0; a < OR_NPOP; ++a) {
        int64_t n = (int64_t)floor(p->full_size[a] * scale + 0.5);
        if (n < 1) n = 1;
        nt->pop_size[a] = (int32_t)n;
        nt->pop_off[a + 1] = nt->pop_off[a] + (int32_t)n;
    }
    nt->N = nt->pop_off[OR_NPOP];

    /* Synapse counts per ordered pair (a -> b). */
    int64_t K[64], base[65];
    base[0] = 0;
    for (int a = 0; a < OR_NPOP; ++a)
        for (int b = 0; b < OR_NPOP; ++b) {
            double pr = conn[8 * a + b];
            int64_t k = 0;
            if (pr > 0.0) {
                double pairs = (double)nt->pop_size[a] * (double)nt->pop_size[b];
                k = llround(log1p(-pr) / log1p(-1.0 / pairs));
            }
            K[8 * a + b] = k;
            base[8 * a + b + 1] = base[8 * a + b] + k;
        }
    nt->M = base[64];
    const int64_t M = nt->M;

    int32_t *pre = (int32_t *)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
    int32_t *post = (int32_t *)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
    int32_t *wq = (int32_t *)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
    uint8_t *d = (uint8_t *)malloc((size_t)(M ? M : 1));
    double *w64 = p->mode == 1 ? (double *)malloc((size_t)(M ? M : 1) * sizeof(double)) : NULL;
    if (!pre || !post || !wq || !d || (p->mode == 1 && !w64)) {
        free(pre); free(post); free(wq); free(d); free(w64); or_free(nt);
        set_err("out of host memory");
        return NULL;
    }

    const double two_pi = 6.283185307179586;
    int bad = 0;
    for (int a = 0; a < OR_NPOP; ++a)
        for (int b = 0; b < OR_NPOP; ++b) {
            const int64_t Kab = K[8 * a + b];
            const int64_t b0 = base[8 * a + b];
            const int exc = is_exc(a);
            double wm = exc ? p->w_mean_pa : p->g * p->w_mean_pa;
            double ws = exc ? p->w_sd_pa : fabs(p->g) * p->w_sd_pa;
            if (a == 2 && b == 0) wm = p->l4e_l23e_factor * p->w_mean_pa;   /* L4E -> L2/3E */
            const double dm = exc ? p->d_mean_exc_ms : p->d_mean_inh_ms;
            const double ds = exc ? p->d_sd_exc_ms : p->d_sd_inh_ms;
#pragma omp parallel for schedule(static) reduction(| : bad)
            for (int64_t s = 0; s < Kab; ++s) {
                uint64_t c[4] = {(uint64_t)s, (uint64_t)(8 * a + b), 0, TAG_SYN};
                uint64_t k[2] = {seed, 0}, x[4];
                or_philox(c, k, x);
                int32_t i_pre = nt->pop_off[a] + (int32_t)mulhi_n(x[0], nt->pop_size[a]);
                int32_t i_post = nt->pop_off[b] + (int32_t)mulhi_n(x[1], nt->pop_size[b]);
                double r = sqrt(-2.0 * log(u53p(x[2])));
                double phi = two_pi * u53(x[3]);
                double zw = r * cos(phi);
                double zd = r * sin(phi);
                double w = wm + ws * zw;
                if (exc && w < 0.0) w = 0.0;
                if (!exc && w > 0.0) w = 0.0;
                double dd = rint((dm + ds * zd) / p->dt_ms);
                if (dd < 1.0) dd = 1.0;
                if (dd > 255.0) dd = 255.0;
                pre[b0 + s] = i_pre;
                post[b0 + s] = i_post;
                d[b0 + s] = (uint8_t)dd;
                if (w64) w64[b0 + s] = w;
                int32_t q = 0;
                if (quantise(p, w, &q) != 0) bad |= 1;
                wq[b0 + s] = q;
            }
        }
    if (bad) {
        free(pre); free(post); free(wq); free(d); free(w64); or_free(nt);
        set_err("weight out of int32 range");
        return NULL;
    }
    int rc = finish_network(nt, pre, post, wq, w64, d);
    free(pre); free(post); free(wq); free(d); free(w64);
    if (rc) { or_free(nt); return NULL; }
    return nt;
}

/*
 * Build a network from an explicit synapse list (hand-made test networks).
 * pop_size[8] gives the populations (neuron ids ordered by population); the
 * synapse arrays are pre, post, weight (pA, double) and delay (steps, 1..255).
 */
or_net *or_build_explicit(const or_params *p, uint64_t seed, const int32_t *pop_size,
                          int64_t M, const int32_t *pre, const int32_t *post,
                          const double *w, const int32_t *d)
{
    if (check_params(p)) return NULL;
    or_net *nt = new_net(p, seed);
    if (!nt) return NULL;
    nt->pop_off[0] = 0;
    for (int a = 0; a < OR_NPOP; ++a) {
        if (pop_size[a] < 0) { or_free(nt); set_err("negative population size"); return NULL; }
        nt->pop_size[a] = pop_size[a];
        nt->pop_off[a + 1] = nt->pop_off[a] + pop_size[a];
    }
    nt->N = nt->pop_off[OR_NPOP];
    nt->M = M;
    int32_t *wq = (int32_t *)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
    uint8_t *dd = (uint8_t *)malloc((size_t)(M ? M : 1));
    double *w64 = p->mode == 1 ? (double *)malloc((size_t)(M ? M : 1) * sizeof(double)) : NULL;
    if (!wq || !dd || (p->mode == 1 && !w64)) { free(wq); free(dd); free(w64); or_free(nt); set_err("out of host memory"); return NULL; }
    for (int64_t s = 0; s < M; ++s) {
        if (pre[s] < 0 || pre[s] >= nt->N || post[s] < 0 || post[s] >= nt->N || d[s] < 1 || d[s] > 255) {
            free(wq); free(dd); free(w64); or_free(nt); set_err("synapse out of range"); return NULL;
        }
        if (quantise(p, w[s], &wq[s]) != 0) { free(wq); free(dd); free(w64); or_free(nt); set_err("weight out of int32 range"); return NULL; }
        dd[s] = (uint8_t)d[s];
        if (w64) w64[s] = w[s];
    }
    int rc = finish_network(nt, (int32_t *)pre, (int32_t *)post, wq, w64, dd);
    free(wq); free(dd); free(w64);
    if (rc) { or_free(nt); return NULL; }
    return nt;
}

/* ------------------------------------------------------------------------- */
/* Simulation                                                                */
/* ------------------------------------------------------------------------- */
static int poisson_count(const or_net *nt, int pop, int64_t n, int32_t i)
{
    uint64_t c[4] = {(uint64_t)n, (uint64_t)(i / 8), 0, TAG_POIS}, k[2] = {nt->seed, nt->p.pois_stream}, x[4];
    or_philox(c, k, x);
    const int h = i % 8;
    const uint64_t word = x[h / 2];
    uint64_t v = (h % 2 == 0) ? (word >> 32) : (word & 0xFFFFFFFFULL);
    int cnt = 0;
    for (int j = 0; j < OR_KMAX; ++j)
        if (v >= nt->T[pop][j]) cnt++;
    return cnt;
}

int or_poisson_count(const or_net *nt, int64_t n, int32_t i)
{
    if (i < 0 || i >= nt->N) return -1;
    return poisson_count(nt, nt->pop_of[i], n, i);
}

static int record(or_net *nt, int64_t n, int32_t i)
{
    if (nt->nrec == nt->caprec) {
        int64_t cap = nt->caprec ? 2 * nt->caprec : 4096;
        int64_t *s = (int64_t *)realloc(nt->rec_step, (size_t)cap * sizeof(int64_t));
        if (!s) return -1;
        nt->rec_step = s;
        int32_t *q = (int32_t *)realloc(nt->rec_id, (size_t)cap * sizeof(int32_t));
        if (!q) return -1;
        nt->rec_id = q;
        nt->caprec = cap;
    }
    nt->rec_step[nt->nrec] = n;
    nt->rec_id[nt->nrec] = i;
    nt->nrec++;
    return 0;
}

/* One step of every neuron, then delivery of every spike of the step. */
static int step_once(or_net *nt)
{
    const int32_t N = nt->N, R = nt->R;
    const int64_t n = nt->step;
    const int64_t slot = n & (R - 1);
    const int pois = nt->p.poisson_on;
    int64_t npois = 0;

    if (nt->p.mode == 0) {
#pragma omp parallel for schedule(static) reduction(+ : npois)
        for (int32_t i = 0; i < N; ++i) {
            const int pop = nt->pop_of[i];
            int32_t *cell = &nt->ring[slot * N + i];
            int32_t inq = *cell;
            *cell = 0;
            if (pois) {
                int k = poisson_count(nt, pop, n, i);
                npois += k;
                inq += k * nt->wq_ext;
            }
            float in = (float)inq * 0.00390625f;
            float u = nt->uf[i], I = nt->If[i];
            if (nt->refr[i] > 0) {
                nt->refr[i] -= 1;
            } else {
                float a = nt->P22f * u;
                float b = nt->P21f * I;
                u = a + b;
                if (nt->cdc_f[pop] != 0.0f) u = u + nt->cdc_f[pop];
            }
            float c = nt->P11f * I;
            I = c + in;
            uint8_t s = 0;
            if (u > nt->thetaf) {
                s = 1;
                u = 0.0f;
                nt->refr[i] = nt->ref_steps;
            }
            nt->uf[i] = u;
            nt->If[i] = I;
            nt->spk[i] = s;
        }
    } else {
#pragma omp parallel for schedule(static) reduction(+ : npois)
        for (int32_t i = 0; i < N; ++i) {
            const int pop = nt->pop_of[i];
            double *cell = &nt->ringd[slot * N + i];
            double in = *cell;
            *cell = 0.0;
            if (pois) {
                int k = poisson_count(nt, pop, n, i);
                npois += k;
                in = in + (double)k * nt->w_ext;
            }
            double u = nt->ud[i], I = nt->Id[i];
            if (nt->refr[i] > 0) {
                nt->refr[i] -= 1;
            } else {
                u = nt->P22 * u + nt->P21 * I;
                if (nt->cdc_d[pop] != 0.0) u = u + nt->cdc_d[pop];
            }
            I = nt->P11 * I + in;
            uint8_t s = 0;
            if (u > nt->theta) {
                s = 1;
                u = 0.0;
                nt->refr[i] = nt->ref_steps;
            }
            nt->ud[i] = u;
            nt->Id[i] = I;
            nt->spk[i] = s;
        }
    }
    nt->n_pois += npois;

    /* Spikes of this step, in neuron order; delivery into future slots. */
    int32_t S = 0;
    for (int32_t i = 0; i < N; ++i) {
        if (!nt->spk[i]) continue;
        S++;
        if (record(nt, n, i)) { set_err("out of host memory (spike record)"); return -1; }
        const int64_t r0 = nt->row_ptr[i], r1 = nt->row_ptr[i + 1];
        nt->n_events += r1 - r0;
        for (int64_t j = r0; j < r1; ++j) {
            const int64_t at = ((n + nt->d[j]) & (R - 1)) * (int64_t)N + nt->post[j];
            if (nt->p.mode == 0) nt->ring[at] += nt->wq[j];
            else nt->ringd[at] += nt->w64[j];
        }
    }
    nt->n_spikes += S;
    if (S > nt->max_s) nt->max_s = S;
    nt->step = n + 1;
    return 0;
}

/* Deliver the rows of the listed neurons as if they had spiked in the step
   before the current one (external stimulation); not recorded or counted. */
int or_inject(or_net *nt, const int32_t *ids, int64_t count)
{
    const int64_t n = nt->step - 1;
    for (int64_t q = 0; q < count; ++q) {
        const int32_t i = ids[q];
        if (i < 0 || i >= nt->N) { set_err("neuron id out of range"); return -1; }
        for (int64_t j = nt->row_ptr[i]; j < nt->row_ptr[i + 1]; ++j) {
            const int64_t at = ((n + nt->d[j]) & (nt->R - 1)) * (int64_t)nt->N + nt->post[j];
            if (nt->p.mode == 0) nt->ring[at] += nt->wq[j];
            else nt->ringd[at] += nt->w64[j];
        }
    }
    return 0;
}

int or_run(or_net *nt, int64_t steps)
{
    for (int64_t s = 0; s < steps; ++s)
        if (step_once(nt)) return -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Accessors                                                                 */
/* ------------------------------------------------------------------------- */
int32_t or_num_neurons(const or_net *nt) { return nt->N; }
int64_t or_num_synapses(const or_net *nt) { return nt->M; }
int32_t or_ring_depth(const or_net *nt) { return nt->R; }
int64_t or_step(const or_net *nt) { return nt->step; }
int32_t or_wq_ext(const or_net *nt) { return nt->wq_ext; }

void or_pop_offsets(const or_net *nt, int32_t out[OR_NPOP + 1])
{
    memcpy(out, nt->pop_off, sizeof(nt->pop_off));
}

void or_poisson_table(const or_net *nt, int pop, uint64_t out[OR_KMAX])
{
    memcpy(out, nt->T[pop], sizeof(nt->T[pop]));
}

/* out: P22, P11, P21, P20 (double) then their float roundings, then theta. */
void or_constants(const or_net *nt, double out[9])
{
    out[0] = nt->P22; out[1] = nt->P11; out[2] = nt->P21; out[3] = nt->P20;
    out[4] = nt->P22f; out[5] = nt->P11f; out[6] = nt->P21f; out[7] = (float)nt->P20;
    out[8] = nt->theta;
}

void or_get_csr(const or_net *nt, int64_t *row_ptr, int32_t *post, int32_t *wq, uint8_t *d, double *w64)
{
    if (row_ptr) memcpy(row_ptr, nt->row_ptr, ((size_t)nt->N + 1) * sizeof(int64_t));
    if (post) memcpy(post, nt->post, (size_t)nt->M * sizeof(int32_t));
    if (wq) memcpy(wq, nt->wq, (size_t)nt->M * sizeof(int32_t));
    if (d) memcpy(d, nt->d, (size_t)nt->M);
    if (w64 && nt->w64) memcpy(w64, nt->w64, (size_t)nt->M * sizeof(double));
}

void or_get_state(const or_net *nt, double *u, double *I, int32_t *refr)
{
    for (int32_t i = 0; i < nt->N; ++i) {
        if (u) u[i] = nt->p.mode == 0 ? (double)nt->uf[i] : nt->ud[i];
        if (I) I[i] = nt->p.mode == 0 ? (double)nt->If[i] : nt->Id[i];
        if (refr) refr[i] = nt->refr[i];
    }
}

void or_set_state(or_net *nt, const double *u, const double *I, const int32_t *refr)
{
    for (int32_t i = 0; i < nt->N; ++i) {
        if (nt->p.mode == 0) {
            if (u) nt->uf[i] = (float)u[i];
            if (I) nt->If[i] = (float)I[i];
        } else {
            if (u) nt->ud[i] = u[i];
            if (I) nt->Id[i] = I[i];
        }
        if (refr) nt->refr[i] = refr[i];
    }
}

/* Sum of the pending input-buffer contents (Q8 units in mirror mode). */
double or_ring_sum(const or_net *nt)
{
    double s = 0.0;
    const int64_t cells = (int64_t)nt->R * nt->N;
    for (int64_t q = 0; q < cells; ++q) s += nt->p.mode == 0 ? (double)nt->ring[q] : nt->ringd[q];
    return s;
}

int64_t or_num_recorded(const or_net *nt) { return nt->nrec; }

void or_get_spikes(const or_net *nt, int64_t *steps, int32_t *ids)
{
    memcpy(steps, nt->rec_step, (size_t)nt->nrec * sizeof(int64_t));
    memcpy(ids, nt->rec_id, (size_t)nt->nrec * sizeof(int32_t));
}

void or_clear_spikes(or_net *nt) { nt->nrec = 0; }

/* out: steps, spikes, recurrent events, Poisson events, max spikes per step */
void or_get_counters(const or_net *nt, int64_t out[5])
{
    out[0] = nt->step; out[1] = nt->n_spikes; out[2] = nt->n_events;
    out[3] = nt->n_pois; out[4] = nt->max_s;
}
