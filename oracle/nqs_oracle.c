/*
 * nqs_oracle.c -- CPU FP64 oracle for mixed-precision NQS sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * library never links, includes or calls it, and it shares no code with it.
 *
 * Everything is written from the definitions in the paper
 * "Neural Quantum States in Mixed Precision" (arXiv 2601.20782):
 *   - amplitudes / sampling target:      Sec. II, Eq. (1) and Eq. (eq:loss)
 *   - MH acceptance alpha = min(1, s):   Sec. III.A, Eq. (eq: unperturbed acceptance rate)
 *   - single-bit-flip proposal q = 1/n:  App. C, Eq. (eq:app:local_prop)
 *   - exchange (swap) proposal:          App. E
 *   - TFIM and Heisenberg Hamiltonians:  Eq. (eq:TFIM), App. E
 *   - RBM log-amplitude:                 App. G
 *   - local energies:                    App. I.1, Eq. (eq:local_energies)
 *   - forces and O_k:                    App. I.1, Eq. (eq:forces)
 *   - S matrix:                          App. I.2, Eq. (eq:smat)
 *   - reduced-precision formats:         App. A, Table A
 * No blocking, fusion or incremental state: every log-amplitude is a full
 * forward pass, every sum a plain loop, in FP64.
 *
 * The parallelism is OpenMP over independent chains / samples only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* dtype codes (same numbering as the public interface, chosen independently) */
enum { ORC_F64 = 0, ORC_F32 = 1, ORC_F16 = 2, ORC_BF16 = 3, ORC_E4M3 = 4 };
enum { ORC_RBM = 0, ORC_FFNN = 1, ORC_TABLE = 2 };
enum { ORC_FLIP = 0, ORC_EXCHANGE = 1 };
enum { ORC_TFIM = 0, ORC_HEIS = 1 };

#define ORC_MAX_LAYERS 8

typedef struct {
    int32_t arch;                 /* ORC_RBM / ORC_FFNN / ORC_TABLE */
    int32_t n_visible;            /* N */
    int32_t n_layers;             /* RBM: 1 (M = widths[0]); FFNN: number of dense layers */
    int32_t widths[ORC_MAX_LAYERS];
    int32_t act_dtype;            /* FFNN: format the inputs of layers >= 2 are rounded to */
    int32_t marshall;             /* 1: psi carries the Marshall sign (-1)^{#up on sublattice A} */
    int32_t lat_dim, lat_L;       /* lattice used by the Marshall sublattice */
    double act_scale[ORC_MAX_LAYERS]; /* E4M3 only: per-layer activation scales (value = q*scale) */
    const double *params;         /* parameter vector (already rounded when emulating a format) */
    const double *table_logamp;   /* ORC_TABLE: log|psi(x)| for x = 0..2^N-1 */
    const int8_t *table_sign;     /* ORC_TABLE: sign of psi(x) (+1/-1, 0 = psi(x) == 0) */
} orc_model;

typedef struct {
    int32_t kind;                 /* ORC_TFIM / ORC_HEIS */
    int32_t dim, L, pbc;
    double J, h;
} orc_ham;

typedef struct {
    int64_t n_chains;
    int32_t n_sweeps, n_burnin, sweep_size, move;
    uint64_t seed, step_offset;
    uint32_t instance_id;
    int32_t init_chains;          /* 1: draw initial states from the init stream */
} orc_sample_cfg;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Ten rounds of the */
/* 4x32 Philox S-box with the published multipliers and Weyl key increments. */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The stream layout: key = seed; counter = (step, chain, instance<<8 | tag). */
static void stream_block(uint64_t seed, uint64_t step, uint32_t chain, uint32_t inst, uint32_t tag,
                         uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)step, (uint32_t)(step >> 32), chain, (inst << 8) | tag};
    orc_philox4x32_10(ctr, key, out);
}

/* zeta(x) = sigma g(x) of the noisy target log pi~ = log pi + zeta (Sec. IV.A):
 * g a standard normal fixed per configuration.  Philox4x32-10 with the
 * configuration's 32-bit words as counter (spin i up = bit i % 32 of word i / 32)
 * and the seed as key; Box-Muller (Box and Muller 1958) on the first two
 * outputs: u1 = ((r0 >> 8) + 1) 2^-24 in (0, 1], u2 = (r1 >> 8) 2^-24,
 * g = sqrt(-2 ln u1) cos(2 pi u2).  N <= 128. */
void orc_noise_zeta(const int8_t *configs, int64_t n, int32_t N, double sigma, uint64_t seed, double *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t k = 0; k < n; ++k) {
        uint32_t w[4] = {0u, 0u, 0u, 0u}, r[4];
        for (int32_t i = 0; i < N && i < 128; ++i)
            if (configs[k * N + i] > 0) w[i >> 5] |= 1u << (i & 31);
        orc_philox4x32_10(w, key, r);
        const double u1 = (double)((r[0] >> 8) + 1u) / 16777216.0;
        const double u2 = (double)(r[1] >> 8) / 16777216.0;
        out[k] = sigma * sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
    }
}

/* uniform index in [0, n) from a 32-bit word: floor(r * n / 2^32) */
static int32_t index_from_word(uint32_t r, int32_t n)
{
    return (int32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

/* u in [0,1) on the 2^-24 grid (exactly representable in FP32 and FP64) */
static double uniform_from_word(uint32_t r)
{
    return (double)(r >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision formats (App. A, Table A).  Round-to-nearest-even of an */
/* FP64 value straight to the target format (one rounding), by definition:  */
/* the value is scaled by its quantum 2^(E-p+1) and rounded to an integer.   */
/* ------------------------------------------------------------------------ */
static double round_to_format(double x, int p, int emin, double maxfinite, int inf_on_overflow)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);            /* x = m * 2^e, 0.5 <= |m| < 1  ->  unbiased exponent e-1 */
    int E = e - 1;
    if (E < emin) E = emin;        /* subnormal range: fixed quantum */
    double q = ldexp(1.0, E - (p - 1));
    double r = nearbyint(x / q) * q;  /* x/q is exact (power-of-two scaling); default mode = RNE */
    if (fabs(r) > maxfinite) return inf_on_overflow ? copysign(INFINITY, x) : NAN;
    return r;
}

double orc_round(double x, int32_t dtype)
{
    switch (dtype) {
    case ORC_F64: return x;
    case ORC_F32: return (double)(float)x;                              /* IEEE binary32 */
    case ORC_F16: return round_to_format(x, 11, -14, 65504.0, 1);      /* IEEE binary16 */
    case ORC_BF16: return round_to_format(x, 8, -126, ldexp(255.0, 120), 1); /* bfloat16 */
    case ORC_E4M3: return round_to_format(x, 4, -6, 448.0, 0);         /* OCP FP8 E4M3 (no inf) */
    default: return NAN;
    }
}

void orc_round_array(const double *x, int64_t n, int32_t dtype, double *out)
{
#pragma omp parallel for schedule(static) if (n > 65536)
    for (int64_t k = 0; k < n; ++k) out[k] = orc_round(x[k], dtype);
}

/* ------------------------------------------------------------------------ */
/* Lattice: sites i = x*L + y (2D) or i (1D); nearest-neighbour bonds        */
/* <i,j> (Eq. eq:TFIM, App. E).  Periodic wrap when pbc.                     */
/* ------------------------------------------------------------------------ */
int32_t orc_bonds(int32_t dim, int32_t L, int32_t pbc, int32_t *out_pairs)
{
    int32_t nb = 0;
    if (dim == 1) {
        for (int32_t i = 0; i < L; ++i) {
            int32_t j = i + 1;
            if (j == L) { if (!pbc) continue; j = 0; }
            if (out_pairs) { out_pairs[2 * nb] = i; out_pairs[2 * nb + 1] = j; }
            ++nb;
        }
        return nb;
    }
    for (int32_t x = 0; x < L; ++x)
        for (int32_t y = 0; y < L; ++y) {
            int32_t i = x * L + y;
            /* neighbour along x */
            if (x + 1 < L || pbc) {
                int32_t j = ((x + 1) % L) * L + y;
                if (out_pairs) { out_pairs[2 * nb] = i; out_pairs[2 * nb + 1] = j; }
                ++nb;
            }
            /* neighbour along y */
            if (y + 1 < L || pbc) {
                int32_t j = x * L + (y + 1) % L;
                if (out_pairs) { out_pairs[2 * nb] = i; out_pairs[2 * nb + 1] = j; }
                ++nb;
            }
        }
    return nb;
}

/* sublattice A: (x+y) even in 2D, i even in 1D */
static int on_sublattice_a(int32_t dim, int32_t L, int32_t i)
{
    if (dim == 1) return (i % 2) == 0;
    return ((i / L + i % L) % 2) == 0;
}

/* Marshall sign (-1)^{number of up spins on sublattice A} */
static int marshall_sign(const orc_model *m, const int8_t *s)
{
    int up = 0;
    for (int32_t i = 0; i < m->n_visible; ++i)
        if (s[i] > 0 && on_sublattice_a(m->lat_dim, m->lat_L, i)) ++up;
    return (up % 2) ? -1 : 1;
}

/* ------------------------------------------------------------------------ */
/* Networks.  log cosh written in the overflow-safe form                     */
/*   log cosh z = |z| + log(1 + exp(-2|z|)) - log 2.                         */
/* ------------------------------------------------------------------------ */
static double logcosh(double z)
{
    double a = fabs(z);
    return a + log1p(exp(-2.0 * a)) - 0.69314718055994530942;   /* log 2 */
}

/* RBM (App. G) with real parameters: f(s) = a.s + sum_j logcosh((W s + b)_j) */
static double rbm_logamp(const orc_model *m, const int8_t *s)
{
    const int32_t N = m->n_visible, M = m->widths[0];
    const double *a = m->params, *b = a + N, *W = b + M;
    double f = 0.0;
    for (int32_t i = 0; i < N; ++i) f += a[i] * s[i];
    for (int32_t j = 0; j < M; ++j) {
        double th = b[j];
        for (int32_t i = 0; i < N; ++i) th += W[(int64_t)j * N + i] * s[i];
        f += logcosh(th);
    }
    return f;
}

/* round a layer input to the activation format (per-layer scale for E4M3) */
static double round_act(const orc_model *m, int layer, double v)
{
    if (m->act_dtype == ORC_E4M3) {
        double sc = m->act_scale[layer];
        return orc_round(v / sc, ORC_E4M3) * sc;
    }
    return orc_round(v, m->act_dtype);
}

/* Dense network: h_l = ReLU(W_l h_{l-1} + b_l) for l < L; f = sum_k logcosh(z_L,k).
 * When emulating a reduced format, each layer's input (h_{l-1}, l >= 2) is
 * rounded to act_dtype because it is an operand of a matrix product. */
static double ffnn_forward(const orc_model *m, const int8_t *s, double **acts /* optional, per layer pre-activations */)
{
    const int32_t N = m->n_visible, nl = m->n_layers;
    int32_t maxw = N;
    for (int l = 0; l < nl; ++l) if (m->widths[l] > maxw) maxw = m->widths[l];
    double *in = (double *)malloc(sizeof(double) * maxw);
    double *out = (double *)malloc(sizeof(double) * maxw);
    for (int32_t i = 0; i < N; ++i) in[i] = s[i];
    const double *p = m->params;
    int32_t prev = N;
    double f = 0.0;
    for (int l = 0; l < nl; ++l) {
        const int32_t w = m->widths[l];
        const double *W = p, *b = p + (int64_t)w * prev;
        for (int32_t k = 0; k < w; ++k) {
            double z = b[k];
            for (int32_t i = 0; i < prev; ++i) z += W[(int64_t)k * prev + i] * in[i];
            out[k] = z;
        }
        if (acts) memcpy(acts[l], out, sizeof(double) * w);
        p = b + w;
        if (l == nl - 1) {
            for (int32_t k = 0; k < w; ++k) f += logcosh(out[k]);
        } else {
            for (int32_t k = 0; k < w; ++k) {
                double h = out[k] > 0.0 ? out[k] : 0.0;
                in[k] = round_act(m, l + 1, h);
            }
            prev = w;
        }
    }
    free(in);
    free(out);
    return f;
}

static uint64_t table_index(int32_t N, const int8_t *s)
{
    uint64_t x = 0;
    for (int32_t i = 0; i < N; ++i) if (s[i] > 0) x |= (uint64_t)1 << i;
    return x;
}

/* log|psi(s)| and the sign of psi(s) (Sec. II: the network outputs log psi). */
double orc_logamp(const orc_model *m, const int8_t *s, int32_t *sign_out)
{
    double f;
    int sign = 1;
    switch (m->arch) {
    case ORC_RBM: f = rbm_logamp(m, s); break;
    case ORC_FFNN: f = ffnn_forward(m, s, NULL); break;
    case ORC_TABLE: {
        uint64_t x = table_index(m->n_visible, s);
        f = m->table_logamp[x];
        sign = m->table_sign[x];
        break;
    }
    default: f = NAN;
    }
    if (m->marshall) sign *= marshall_sign(m, s);
    if (sign_out) *sign_out = sign;
    return f;
}

void orc_logamp_batch(const orc_model *m, const int8_t *samples, int64_t n, double *out, int32_t *signs)
{
    const int32_t N = m->n_visible;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        int32_t sg;
        out[k] = orc_logamp(m, samples + k * N, &sg);
        if (signs) signs[k] = sg;
    }
}

/* ------------------------------------------------------------------------ */
/* Chain initialisation from the init stream (tag 1).  Word w of the stream  */
/* is component w%4 of block w/4.                                            */
/* ------------------------------------------------------------------------ */
static uint32_t init_word(uint64_t seed, uint32_t chain, uint32_t inst, uint32_t w)
{
    uint32_t blk[4];
    stream_block(seed, (uint64_t)(w / 4), chain, inst, 1u, blk);
    return blk[w % 4];
}

void orc_init_chain(int32_t N, int32_t move, uint64_t seed, uint32_t chain, uint32_t inst, int8_t *s)
{
    if (move == ORC_FLIP) {
        /* independent uniform spins: bit i%32 of word i/32 */
        for (int32_t i = 0; i < N; ++i) {
            uint32_t w = init_word(seed, chain, inst, (uint32_t)(i / 32));
            s[i] = ((w >> (i % 32)) & 1u) ? 1 : -1;
        }
    } else {
        /* zero magnetisation: N/2 up then N/2 down, shuffled by Fisher-Yates
         * (for k = N-1 .. 1 swap s[k] with s[floor(r_m (k+1) / 2^32)], m = N-1-k). */
        for (int32_t i = 0; i < N; ++i) s[i] = (i < N / 2) ? 1 : -1;
        for (int32_t k = N - 1; k >= 1; --k) {
            uint32_t r = init_word(seed, chain, inst, (uint32_t)(N - 1 - k));
            int32_t j = index_from_word(r, k + 1);
            int8_t t = s[k]; s[k] = s[j]; s[j] = t;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Metropolis-Hastings (Sec. III.A): propose y ~ q(.|x), accept with         */
/* probability min(1, exp(log p(y) - log p(x))), log p = 2 log|psi| (Sec. II).*/
/* One Philox block per proposal: site i from r0, partner j from r1          */
/* (exchange), u from r2.  A sweep is sweep_size proposals; after n_burnin   */
/* sweeps one sample per chain per sweep is kept.                            */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t i, j; double u; uint32_t ubits; } proposal;

static proposal make_proposal(uint64_t seed, uint64_t step, uint32_t chain, uint32_t inst, int32_t N, int32_t move)
{
    uint32_t r[4];
    stream_block(seed, step, chain, inst, 0u, r);
    proposal p;
    p.i = index_from_word(r[0], N);
    p.j = -1;
    if (move == ORC_EXCHANGE) {
        int32_t j = index_from_word(r[1], N - 1);
        if (j >= p.i) j += 1;
        p.j = j;
    }
    p.ubits = r[2] >> 8;
    p.u = uniform_from_word(r[2]);
    return p;
}

static void apply_move(int8_t *s, const proposal *p)
{
    if (p->j < 0) { s[p->i] = (int8_t)-s[p->i]; return; }
    int8_t t = s[p->i]; s[p->i] = s[p->j]; s[p->j] = t;
}

/* accept iff u < exp(min(Delta, 0)) */
static int mh_accept(double delta, double u)
{
    if (!(delta == delta)) return 0;   /* non-finite ratio rejects */
    double a = delta < 0.0 ? exp(delta) : 1.0;
    return u < a;
}

int32_t orc_sample(const orc_model *m, const orc_sample_cfg *cfg, int8_t *chain_state,
                   int8_t *samples, double *logpsi, uint64_t *n_accepted)
{
    const int32_t N = m->n_visible;
    const int32_t sw = cfg->sweep_size > 0 ? cfg->sweep_size : N;
    const int64_t C = cfg->n_chains;
    const int64_t total = (int64_t)(cfg->n_burnin + cfg->n_sweeps) * sw;
    if (cfg->move == ORC_EXCHANGE && N < 2) return 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        int8_t *s = chain_state + c * N;
        int8_t *y = (int8_t *)malloc((size_t)N);
        if (cfg->init_chains) orc_init_chain(N, cfg->move, cfg->seed, (uint32_t)c, cfg->instance_id, s);
        double f = orc_logamp(m, s, NULL);
        uint64_t acc = 0;
        for (int64_t k = 0; k < total; ++k) {
            proposal p = make_proposal(cfg->seed, cfg->step_offset + (uint64_t)k, (uint32_t)c,
                                       cfg->instance_id, N, cfg->move);
            memcpy(y, s, (size_t)N);
            apply_move(y, &p);
            double fy = orc_logamp(m, y, NULL);   /* full forward, no incremental state */
            double delta = 2.0 * (fy - f);
            if (mh_accept(delta, p.u)) { memcpy(s, y, (size_t)N); f = fy; ++acc; }
            if ((k + 1) % sw == 0) {
                int64_t sweep = (k + 1) / sw - 1 - cfg->n_burnin;
                if (sweep >= 0) {
                    if (samples) memcpy(samples + (sweep * C + c) * N, s, (size_t)N);
                    if (logpsi) logpsi[sweep * C + c] = f;
                }
            }
        }
        if (n_accepted) n_accepted[c] = acc;
        free(y);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Decision replay.  A device run reports, for each traced chain and step,   */
/* the site pair, the u bits, its own Delta and its decision.  The oracle    */
/* re-derives site, partner and u from its own generator (must agree bit for */
/* bit), evaluates Delta in FP64 on the same pre-move state, and checks the  */
/* decision; decisions may differ only where |log u - Delta| <= tau.  The    */
/* device's decision is then applied so both stay on one trajectory.         */
/* stats: [0] site/u mismatches, [1] decisions differing beyond tau,         */
/*        [2] near ties (|log u - Delta| <= tau), [3] decisions equal,       */
/*        [4] max |Delta_dev - Delta_64| on steps that changed the state     */
/* ------------------------------------------------------------------------ */
void orc_replay(const orc_model *m, const orc_sample_cfg *cfg, int64_t n_traced, const int32_t *chain_ids,
                const int8_t *start_states, int64_t n_steps, const int32_t *tr_site, const uint32_t *tr_ubits,
                const float *tr_delta, const uint8_t *tr_acc, double tau_rel, int8_t *end_states, double *stats)
{
    const int32_t N = m->n_visible;
    double st[5] = {0, 0, 0, 0, 0};
#pragma omp parallel
    {
        double loc[5] = {0, 0, 0, 0, 0};
        int8_t *s = (int8_t *)malloc((size_t)N);
        int8_t *y = (int8_t *)malloc((size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < n_traced; ++t) {
            const uint32_t c = (uint32_t)chain_ids[t];
            memcpy(s, start_states + t * N, (size_t)N);
            double f = orc_logamp(m, s, NULL);
            for (int64_t k = 0; k < n_steps; ++k) {
                const int64_t idx = t * n_steps + k;
                proposal p = make_proposal(cfg->seed, cfg->step_offset + (uint64_t)k, c, cfg->instance_id, N, cfg->move);
                int32_t dev_i = tr_site[idx] & 0xFFFF, dev_j = (int32_t)((uint32_t)tr_site[idx] >> 16);
                int32_t ref_j = p.j < 0 ? 0xFFFF : p.j;
                if (dev_i != p.i || dev_j != ref_j || tr_ubits[idx] != p.ubits) loc[0] += 1;
                memcpy(y, s, (size_t)N);
                apply_move(y, &p);
                double fy = orc_logamp(m, y, NULL);
                double delta = 2.0 * (fy - f);
                int ref = mh_accept(delta, p.u);
                int dev = tr_acc[idx] != 0;
                double tau = tau_rel * fmax(1.0, fmax(fabs(f), fabs(fy)));
                double gap = fabs(log(p.u) - delta);
                if (p.u == 0.0) gap = INFINITY;
                if (gap <= tau) loc[2] += 1;
                if (ref == dev) loc[3] += 1;
                else if (gap > tau) loc[1] += 1;
                if (memcmp(y, s, (size_t)N) != 0) {
                    double d = fabs((double)tr_delta[idx] - delta);
                    if (d > loc[4]) loc[4] = d;
                }
                if (dev) { memcpy(s, y, (size_t)N); f = fy; }
            }
            if (end_states) memcpy(end_states + t * N, s, (size_t)N);
        }
#pragma omp critical
        {
            for (int q = 0; q < 4; ++q) st[q] += loc[q];
            if (loc[4] > st[4]) st[4] = loc[4];
        }
        free(s);
        free(y);
    }
    for (int q = 0; q < 5; ++q) stats[q] = st[q];
}

/* ------------------------------------------------------------------------ */
/* Local energies (App. I.1, Eq. eq:local_energies):                         */
/*   eps(x) = sum_{x' in C(x)} H(x,x') psi(x')/psi(x).                       */
/* TFIM (Eq. eq:TFIM): H = J sum_<ij> sz sz + h sum_i sx                     */
/*   -> diagonal J sum s_i s_j, off-diagonal h for every single flip.        */
/* Heisenberg (App. E, Pauli matrices): H = J sum_<ij> sigma_i . sigma_j     */
/*   -> diagonal J sum s_i s_j; sx sx + sy sy maps |up,down> to 2|down,up>,  */
/*      so every antiparallel bond contributes 2J psi(x^{ij})/psi(x).        */
/* Sums in FP64.                                                             */
/* ------------------------------------------------------------------------ */
static double psi_ratio(const orc_model *m, const int8_t *y, double f, int32_t sign)
{
    int32_t sy;
    double fy = orc_logamp(m, y, &sy);
    if (sy == 0) return 0.0;
    return (double)(sy * sign) * exp(fy - f);
}

void orc_local_energy(const orc_model *m, const orc_ham *H, const int8_t *samples, int64_t n, double *eloc)
{
    const int32_t N = m->n_visible;
    const int32_t nb = orc_bonds(H->dim, H->L, H->pbc, NULL);
    int32_t *bonds = (int32_t *)malloc(sizeof(int32_t) * 2 * (nb > 0 ? nb : 1));
    orc_bonds(H->dim, H->L, H->pbc, bonds);
#pragma omp parallel
    {
        int8_t *y = (int8_t *)malloc((size_t)N);
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < n; ++k) {
            const int8_t *s = samples + k * N;
            int32_t sign;
            double f = orc_logamp(m, s, &sign);
            double e = 0.0;
            for (int32_t b = 0; b < nb; ++b) e += H->J * s[bonds[2 * b]] * s[bonds[2 * b + 1]];
            if (H->kind == ORC_TFIM) {
                for (int32_t i = 0; i < N; ++i) {
                    memcpy(y, s, (size_t)N);
                    y[i] = (int8_t)-y[i];
                    e += H->h * psi_ratio(m, y, f, sign);
                }
            } else {
                for (int32_t b = 0; b < nb; ++b) {
                    int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
                    if (s[i] == s[j]) continue;
                    memcpy(y, s, (size_t)N);
                    y[i] = s[j]; y[j] = s[i];
                    e += 2.0 * H->J * psi_ratio(m, y, f, sign);
                }
            }
            eloc[k] = e;
        }
        free(y);
    }
    free(bonds);
}

/* ------------------------------------------------------------------------ */
/* Log-derivatives O_k(x) = d log psi(x) / d theta_k (App. I.1, Eq.          */
/* eq:forces; real parameters so O* = O).                                    */
/* RBM: O_a = s, O_b = tanh(theta), O_W[j][i] = tanh(theta_j) s_i.           */
/* FFNN: reverse-mode chain rule written out layer by layer (ReLU'(0) = 0).  */
/* ------------------------------------------------------------------------ */
int64_t orc_num_params(const orc_model *m)
{
    const int32_t N = m->n_visible;
    if (m->arch == ORC_RBM) return (int64_t)N + m->widths[0] + (int64_t)m->widths[0] * N;
    if (m->arch == ORC_FFNN) {
        int64_t p = 0, prev = N;
        for (int l = 0; l < m->n_layers; ++l) { p += (int64_t)m->widths[l] * (prev + 1); prev = m->widths[l]; }
        return p;
    }
    return 0;
}

static void rbm_grad(const orc_model *m, const int8_t *s, double *O)
{
    const int32_t N = m->n_visible, M = m->widths[0];
    const double *b = m->params + N, *W = b + M;
    for (int32_t i = 0; i < N; ++i) O[i] = s[i];
    for (int32_t j = 0; j < M; ++j) {
        double th = b[j];
        for (int32_t i = 0; i < N; ++i) th += W[(int64_t)j * N + i] * s[i];
        double t = tanh(th);
        O[N + j] = t;
        for (int32_t i = 0; i < N; ++i) O[N + M + (int64_t)j * N + i] = t * s[i];
    }
}

static void ffnn_grad(const orc_model *m, const int8_t *s, double *O)
{
    const int32_t N = m->n_visible, nl = m->n_layers;
    double *z[ORC_MAX_LAYERS];
    double *in[ORC_MAX_LAYERS];   /* input vector of each layer (as used in the forward) */
    int32_t prevw[ORC_MAX_LAYERS];
    int32_t prev = N;
    for (int l = 0; l < nl; ++l) {
        z[l] = (double *)malloc(sizeof(double) * m->widths[l]);
        in[l] = (double *)malloc(sizeof(double) * prev);
        prevw[l] = prev;
        prev = m->widths[l];
    }
    ffnn_forward(m, s, z);
    for (int32_t i = 0; i < N; ++i) in[0][i] = s[i];
    for (int l = 1; l < nl; ++l)
        for (int32_t k = 0; k < m->widths[l - 1]; ++k) {
            double h = z[l - 1][k] > 0.0 ? z[l - 1][k] : 0.0;
            in[l][k] = round_act(m, l, h);
        }
    /* offsets of W_l, b_l in the parameter vector */
    int64_t offW[ORC_MAX_LAYERS], offb[ORC_MAX_LAYERS], off = 0;
    for (int l = 0; l < nl; ++l) {
        offW[l] = off; off += (int64_t)m->widths[l] * prevw[l];
        offb[l] = off; off += m->widths[l];
    }
    /* delta_L = d f / d z_L = tanh(z_L) */
    int32_t wl = m->widths[nl - 1];
    double *delta = (double *)malloc(sizeof(double) * wl);
    for (int32_t k = 0; k < wl; ++k) delta[k] = tanh(z[nl - 1][k]);
    for (int l = nl - 1; l >= 0; --l) {
        const int32_t w = m->widths[l], pw = prevw[l];
        for (int32_t k = 0; k < w; ++k) {
            O[offb[l] + k] = delta[k];
            for (int32_t i = 0; i < pw; ++i) O[offW[l] + (int64_t)k * pw + i] = delta[k] * in[l][i];
        }
        if (l == 0) break;
        /* back through W_l and the ReLU of layer l-1 */
        const double *W = m->params + offW[l];
        double *nd = (double *)malloc(sizeof(double) * pw);
        for (int32_t i = 0; i < pw; ++i) {
            double g = 0.0;
            for (int32_t k = 0; k < w; ++k) g += W[(int64_t)k * pw + i] * delta[k];
            nd[i] = z[l - 1][i] > 0.0 ? g : 0.0;
        }
        free(delta);
        delta = nd;
    }
    free(delta);
    for (int l = 0; l < nl; ++l) { free(z[l]); free(in[l]); }
}

void orc_logpsi_grad(const orc_model *m, const int8_t *samples, int64_t n, double *logpsi, double *O)
{
    const int32_t N = m->n_visible;
    const int64_t P = orc_num_params(m);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) {
        const int8_t *s = samples + k * N;
        if (logpsi) logpsi[k] = orc_logamp(m, s, NULL);
        if (O) {
            if (m->arch == ORC_RBM) rbm_grad(m, s, O + k * P);
            else if (m->arch == ORC_FFNN) ffnn_grad(m, s, O + k * P);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* FP64 averages.  E = mean eps (Eq. eq:loss, Monte Carlo estimate); the     */
/* error bar is the standard error of the per-chain means (chains are        */
/* independent).  Samples are laid out [sweep][chain].                       */
/* stats: mean, unbiased variance, stderr of chain means, n.                 */
/* ------------------------------------------------------------------------ */
void orc_stats(const double *eloc, int64_t n, int64_t n_chains, double *stats)
{
    double sum = 0.0;
    for (int64_t k = 0; k < n; ++k) sum += eloc[k];
    const double mean = sum / (double)n;
    double ss = 0.0;
    for (int64_t k = 0; k < n; ++k) ss += (eloc[k] - mean) * (eloc[k] - mean);
    double se = NAN;
    if (n_chains > 1 && n % n_chains == 0) {
        const int64_t per = n / n_chains;
        double cs = 0.0;
        for (int64_t c = 0; c < n_chains; ++c) {
            double cm = 0.0;
            for (int64_t t = 0; t < per; ++t) cm += eloc[t * n_chains + c];
            cm /= (double)per;
            cs += (cm - mean) * (cm - mean);
        }
        se = sqrt(cs / (double)(n_chains - 1) / (double)n_chains);
    }
    stats[0] = mean;
    stats[1] = n > 1 ? ss / (double)(n - 1) : 0.0;
    stats[2] = se;
    stats[3] = (double)n;
}

/* Weighted mean helper: weights w (NULL = every sample weighs 1/n). */
static double wsum(const double *w, int64_t n)
{
    if (!w) return (double)n;
    double t = 0.0;
    for (int64_t k = 0; k < n; ++k) t += w[k];
    return t;
}
#define WK(w, k) ((w) ? (w)[k] : 1.0)

/* Forces F_k = E[O_k eps] - E[O_k] E[eps] (Eq. eq:forces), plain loops in FP64.
 * E is the sample mean, or the w-weighted mean when weights are given
 * (weights = pi(x) over an enumerated space give the exact expectation). */
void orc_forces(const double *O, const double *eloc, const double *w, int64_t n, int64_t P, double *F)
{
    const double W = wsum(w, n);
    double em = 0.0;
    for (int64_t k = 0; k < n; ++k) em += WK(w, k) * eloc[k];
    em /= W;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double a = 0.0, b = 0.0;
        for (int64_t k = 0; k < n; ++k) { a += WK(w, k) * O[k * P + p] * eloc[k]; b += WK(w, k) * O[k * P + p]; }
        F[p] = a / W - (b / W) * em;
    }
}

/* S_pq = E[O_p O_q] - E[O_p] E[O_q] (Eq. eq:smat), plain loops in FP64. */
void orc_smatrix(const double *O, const double *w, int64_t n, int64_t P, double *S)
{
    const double W = wsum(w, n);
    double *mean = (double *)calloc((size_t)P, sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        for (int64_t p = 0; p < P; ++p) mean[p] += WK(w, k) * O[k * P + p];
    for (int64_t p = 0; p < P; ++p) mean[p] /= W;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t p = 0; p < P; ++p)
        for (int64_t q = 0; q < P; ++q) {
            double a = 0.0;
            for (int64_t k = 0; k < n; ++k) a += WK(w, k) * O[k * P + p] * O[k * P + q];
            S[p * P + q] = a / W - mean[p] * mean[q];
        }
    free(mean);
}

/* Sample-space Gram matrix T_kl = (1/n) sum_p Obar_kp Obar_lp, Obar = O - E[O]
 * (the same centred contraction as S, taken over parameters instead of samples). */
void orc_tmatrix(const double *O, int64_t n, int64_t P, double *T)
{
    double *mean = (double *)calloc((size_t)P, sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        for (int64_t p = 0; p < P; ++p) mean[p] += O[k * P + p];
    for (int64_t p = 0; p < P; ++p) mean[p] /= (double)n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n; ++k)
        for (int64_t l = 0; l < n; ++l) {
            double a = 0.0;
            for (int64_t p = 0; p < P; ++p) a += (O[k * P + p] - mean[p]) * (O[l * P + p] - mean[p]);
            T[k * n + l] = a / (double)n;
        }
    free(mean);
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
