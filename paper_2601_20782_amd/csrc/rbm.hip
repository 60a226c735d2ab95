// RBM kernels (App. G, real parameters):  log psi(s) = a.s + sum_j log cosh(theta_j),
// theta = W s + b.
//
// The single-flip ratio uses the cosh addition formula: flipping site i moves
// theta_j to theta_j - 2 s_i W_ji, and
//     cosh(theta - d) / cosh(theta) = cosh d - tanh(theta) sinh d,
// so with per-(i,j) tables C = cosh 2W_ji, S = sinh 2W_ji (built once per
// parameter update from the format-rounded weights) a proposal costs one FMA
// and one multiply per hidden unit:
//     log psi(s') - log psi(s) = -2 a_i s_i + log prod_j (C_ij - s_i t_j S_ij),  t = tanh theta.
// After an accepted flip t_j is advanced with the tanh addition formula,
//     t_j' = (t_j C_ij - s_i S_ij) / r_ij,
// and t is recomputed from theta = W s + b at sweep ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"
#include "internal.h"

namespace nqs {

// ---------------------------------------------------------------------------
// Copy builder: round the FP64 master to `dtype` and derive the tables.
// ---------------------------------------------------------------------------
__global__ void rbm_build_kernel(const double *__restrict__ master, const float *__restrict__ pre, int N, int M,
                                 int dtype, float *a, float *a2, float *b, float *Wt, float2 *CS, float2 *CSt,
                                 unsigned int *max_abs_bits)
{
    const int64_t P = (int64_t)N + M + (int64_t)M * N;
    if (blockIdx.x == 0 && threadIdx.x == 0) CS[(int64_t)N * M] = make_float2(1.0f, 0.0f);   // neutral entry
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        // FP8 values come pre-rounded with their per-tensor scales
        const double v = pre ? (double)pre[p] : round_to_dtype(master[p], dtype);
        if (p < N) {
            a[p] = (float)v;
            a2[p] = (float)(4.0 * v / 0.69314718055994530942);
        } else if (p < N + M) {
            b[p - N] = (float)v;
        } else {
            const int64_t q = p - N - M;
            const int j = (int)(q / N), i = (int)(q % N);
            Wt[(int64_t)i * M + j] = (float)v;
            // tables in FP64, rounded once to FP32
            const float2 cs = make_float2((float)cosh(2.0 * v), (float)sinh(2.0 * v));
            CS[(int64_t)i * M + j] = cs;
            CSt[(int64_t)j * N + i] = cs;
            atomicMax(max_abs_bits, __float_as_uint(fabsf((float)v)));
        }
    }
}

nqs_status rbm_build_copy(nqs_model *m, int dtype, hipStream_t stream)
{
    Copy &c = m->copies[dtype];
    const int N = m->desc.n_visible, M = m->desc.widths[0];
    const size_t nW = (size_t)N * M;
    const size_t P = (size_t)N + M + nW;
    const size_t bytes = sizeof(float) * (2 * N + M + nW) + sizeof(float2) * (2 * nW + 1 + 8 * (size_t)N) + 256 * 10 +
                         (dtype == NQS_FP8_E4M3 ? sizeof(float) * P + 3 * sizeof(unsigned long long) : 0);
    if (!c.block) {
        NQS_HIP_TRY(hipMalloc(&c.block, bytes));
    }
    char *base = (char *)c.block;
    auto carve = [&](size_t sz) {
        char *p = base;
        base += (sz + 255) & ~(size_t)255;
        return p;
    };
    RbmDev &r = c.rbm;
    r.N = N;
    r.M = M;
    r.CS = (float2 *)carve(sizeof(float2) * (nW + 1));
    r.CSt = (float2 *)carve(sizeof(float2) * (nW + 8 * (size_t)N));   // 8 N slack entries for look-ahead loads
    r.Wt = (float *)carve(sizeof(float) * nW);
    r.a = (float *)carve(sizeof(float) * N);
    r.a2 = (float *)carve(sizeof(float) * N);
    r.b = (float *)carve(sizeof(float) * M);
    unsigned int *mx = (unsigned int *)carve(sizeof(unsigned long long));
    float *pre = nullptr;
    unsigned long long *amax = nullptr;
    if (dtype == NQS_FP8_E4M3) {
        pre = (float *)carve(sizeof(float) * P);
        amax = (unsigned long long *)carve(3 * sizeof(unsigned long long));
    }
    if ((size_t)(base - (char *)c.block) > bytes) return set_error(NQS_EDEVICE, "internal layout overflow");
    if (pre) {
        // per-tensor scales for a, b and W (the same tensors the oracle scales)
        const int64_t off[3] = {0, N, (int64_t)N + M}, len[3] = {N, M, (int64_t)nW};
        for (int t = 0; t < 3; ++t) {
            nqs_status e = launch_e4m3_tensor(m->master + off[t], len[t], amax + t, pre + off[t], stream);
            if (e != NQS_OK) return e;
        }
    }
    if (nqs_status z = launch_zero_u64(mx, 1, stream); z != NQS_OK) return z;
    const int blocks = (int)std::min<int64_t>(((int64_t)P + 255) / 256, 4096);
    hipLaunchKernelGGL(rbm_build_kernel, dim3(blocks), dim3(256), 0, stream, m->master, pre, N, M, dtype, r.a, r.a2, r.b,
                       r.Wt, r.CS, r.CSt, mx);
    NQS_HIP_TRY(hipGetLastError());
    unsigned int mbits = 0;
    NQS_HIP_TRY(hipMemcpyAsync(&mbits, mx, sizeof(unsigned int), hipMemcpyDeviceToHost, stream));
    NQS_HIP_TRY(hipStreamSynchronize(stream));
    float mabs;
    std::memcpy(&mabs, &mbits, sizeof(float));
    r.max_abs_w = mabs;
    c.valid = true;
    return NQS_OK;
}

// Largest |W| for which every partial product of 8 ratio factors (each within
// [e^{-2|W|}, e^{2|W|}]) stays inside the FP32 range.
constexpr float kMaxAbsW = 5.0f;

constexpr size_t kLdsBytes = 160 * 1024;

nqs_status rbm_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                      uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream, double noise_sigma,
                      uint64_t noise_seed, unsigned long long *dg_nonfinite, uint32_t *dg_stuck, float *dg_drift)
{
    nqs_status st = ensure_copy(m, cfg.dtype, stream);
    if (st != NQS_OK) return st;
    const RbmDev &net = m->copies[cfg.dtype].rbm;
    if (!std::isfinite(net.max_abs_w)) return set_error(NQS_ENUMERIC, "non-finite weights W in the sampling copy");
    if (!(net.max_abs_w <= kMaxAbsW))
        return set_error(NQS_EUNSUPPORTED, "the product-form RBM sampler needs |W| <= 5");
    const int N = net.N, M = net.M;
    RbmSampleArgs A;
    A.net = net;
    A.chain_state = chain_state;
    A.samples = samples;
    A.logpsi = logpsi;
    A.n_acc = (unsigned long long *)n_accepted;
    A.n_chains = cfg.n_chains;
    A.n_sweeps = cfg.n_sweeps;
    A.n_burnin = cfg.n_burnin;
    A.sweep_size = cfg.sweep_size > 0 ? cfg.sweep_size : N;
    A.refresh_sweeps = cfg.refresh_sweeps > 0 ? cfg.refresh_sweeps : 1;
    A.seed = cfg.seed;
    A.step_offset = cfg.step_offset;
    A.inst = cfg.instance_id;
    A.chain_id_offset = (uint32_t)cfg.chain_id_offset;
    const bool tr = trace && trace->n_chains_traced > 0;
    A.n_traced = tr ? trace->n_chains_traced : 0;
    A.tr_site = tr ? trace->site : nullptr;
    A.tr_ubits = tr ? trace->ubits : nullptr;
    A.tr_delta = tr ? trace->delta : nullptr;
    A.tr_acc = tr ? trace->accepted : nullptr;
    A.noise_sigma = (float)noise_sigma;
    A.noise_key0 = (uint32_t)noise_seed;
    A.noise_key1 = (uint32_t)(noise_seed >> 32);
    const bool diag = dg_drift != nullptr;
    A.dg_nonfinite = diag ? dg_nonfinite : nullptr;
    A.dg_stuck = diag ? dg_stuck : nullptr;
    A.dg_drift = diag ? dg_drift : nullptr;
    const bool noisy = noise_sigma > 0.0;
    if (noisy && (tr || diag || N > 128))
        return set_error(NQS_EUNSUPPORTED, "the noisy sampler takes N <= 128, no trace and no detectors");
    if ((int64_t)(cfg.n_burnin + cfg.n_sweeps) * A.sweep_size == 0) {
        // nothing to propose: only the initial states (and acceptance counts) are defined
        if (cfg.init_chains) {
            st = launch_init_chains(chain_state, cfg.n_chains, N, cfg.move, cfg.seed, cfg.instance_id,
                                    cfg.chain_id_offset, stream);
            if (st != NQS_OK) return st;
        }
        if (n_accepted) return launch_zero_u64(n_accepted, cfg.n_chains, stream);
        return NQS_OK;
    }

    RbmPlan P;
    st = cfg.lanes_per_chain == NQS_LANES_TUNED ? rbm_plan_tuned(m, cfg, nullptr, 0, stream, &P)
                                                : rbm_plan_rule(N, M, cfg.n_chains, cfg.lanes_per_chain, -1, 0, &P);
    if (st != NQS_OK) return st;
    if (noisy && !P.lds) return set_error(NQS_EUNSUPPORTED, "the noisy sampler needs the ratio table in LDS");
    return rbm_launch_plan(A, P, tr || diag, noisy, cfg.init_chains ? 1 : 0, stream);   // detectors run traced
}

// ---------------------------------------------------------------------------
// Run-time detectors: per-chain counters from the traced sampler, reduced to
// the host summary.
// ---------------------------------------------------------------------------
__global__ void diag_zero_kernel(unsigned long long *nf, uint32_t *stuck, float *drift, int64_t C)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
        nf[c] = 0ull;
        stuck[c] = 0u;
        drift[c] = 0.0f;
    }
}

__global__ void __launch_bounds__(256) diag_reduce_kernel(const unsigned long long *nf, const uint32_t *stuck,
                                                          const float *drift, int64_t C, uint32_t stuck_after,
                                                          unsigned long long *out)
{
    __shared__ unsigned long long s_nf[256], s_st[256];
    __shared__ float s_dr[256];
    unsigned long long a = 0, b = 0;
    float d = 0.0f;
    for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
        a += nf[c];
        b += stuck[c] >= stuck_after ? 1ull : 0ull;
        d = fmaxf(d, drift[c]);
    }
    s_nf[threadIdx.x] = a;
    s_st[threadIdx.x] = b;
    s_dr[threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_nf[threadIdx.x] += s_nf[threadIdx.x + w];
            s_st[threadIdx.x] += s_st[threadIdx.x + w];
            s_dr[threadIdx.x] = fmaxf(s_dr[threadIdx.x], s_dr[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s_nf[0];
        out[1] = s_st[0];
        out[2] = (unsigned long long)__float_as_uint(s_dr[0]);
    }
}

nqs_status rbm_sample_checked(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples,
                              float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, nqs_sample_diag *diag,
                              hipStream_t stream)
{
    const int64_t C = cfg.n_chains;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_nf = al(sizeof(unsigned long long) * C), b_st = al(sizeof(uint32_t) * C), b_dr = al(sizeof(float) * C);
    char *ws = (char *)workspace_slot(2, b_nf + b_st + b_dr + 256, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    unsigned long long *nf = diag->nonfinite ? (unsigned long long *)diag->nonfinite : (unsigned long long *)ws;
    uint32_t *st = diag->longest_stuck ? diag->longest_stuck : (uint32_t *)(ws + b_nf);
    float *dr = diag->drift ? diag->drift : (float *)(ws + b_nf + b_st);
    unsigned long long *sum = (unsigned long long *)(ws + b_nf + b_st + b_dr);
    const unsigned zb = (unsigned)std::min<int64_t>((C + 255) / 256, 4096);
    hipLaunchKernelGGL(diag_zero_kernel, dim3(zb), dim3(256), 0, stream, nf, st, dr, C);
    NQS_HIP_TRY(hipGetLastError());
    nqs_status s = rbm_sample(m, cfg, chain_state, samples, logpsi, n_accepted, trace, stream, 0.0, 0, nf, st, dr);
    if (s != NQS_OK) return s;
    const uint32_t k = diag->stuck_after > 0 ? (uint32_t)diag->stuck_after : 10u;
    hipLaunchKernelGGL(diag_reduce_kernel, dim3(1), dim3(256), 0, stream, (const unsigned long long *)nf,
                       (const uint32_t *)st, (const float *)dr, C, k, sum);
    NQS_HIP_TRY(hipGetLastError());
    unsigned long long h[3] = {0, 0, 0};
    NQS_HIP_TRY(hipMemcpyAsync(h, sum, sizeof(h), hipMemcpyDeviceToHost, stream));
    NQS_HIP_TRY(hipStreamSynchronize(stream));
    diag->total_nonfinite = h[0];
    diag->chains_stuck = (int64_t)h[1];
    const uint32_t bits = (uint32_t)h[2];
    std::memcpy(&diag->max_drift, &bits, sizeof(float));
    if (h[0] > 0) return set_error(NQS_ENUMERIC, "non-finite log-ratios in the sampler (proposals rejected)");
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// Launch plans.  The rule: lanes per chain G from (N, M) (16 up to M = 48,
// 32 up to 256, else 64; raised until the spin words and ceil(M/G) units per
// lane fit), the (C,S) table in LDS when it fits in 160 KiB, and as many
// chains per block as spread the chains over every CU.  G fixes the FP32
// summation order of the log-ratio; the other two choices change no result.
// ---------------------------------------------------------------------------
static int kmax_of(int g) { return g == 16 ? 13 : 16; }

nqs_status rbm_plan_rule(int N, int M, int64_t n_chains, int G, int lds_req, int cpb_req, RbmPlan *P)
{
    if (G == 0) G = M > 256 ? 64 : (M > 48 ? 32 : 16);
    else if (G != 16 && G != 32 && G != 64) return set_error(NQS_EINVAL, "lanes_per_chain must be 0, 16, 32 or 64");
    while (G < 64 && ((N + 31) / 32 > G || (M + G - 1) / G > kmax_of(G))) G *= 2;   // spin words and units fit
    if ((N + 31) / 32 > G) return set_error(NQS_EUNSUPPORTED, "too many sites for this many lanes per chain");
    const int K = (M + G - 1) / G;
    if (K > kmax_of(G)) return set_error(NQS_EUNSUPPORTED, "hidden width too large for this many lanes per chain");
    const size_t tab_bytes = sizeof(float2) * ((size_t)N * M + 1);
    const bool fits = tab_bytes <= kLdsBytes;
    const bool lds = lds_req < 0 ? fits : lds_req == 1;
    if (lds && !fits) return set_error(NQS_EUNSUPPORTED, "the ratio table does not fit in LDS");
    // one LDS copy of the table per block; spread the chains over every CU
    const int max_cpb = (G == 16 ? 256 : (G == 32 ? 512 : 1024)) / G;
    const int blocks_per_cu = lds ? (int)std::max<size_t>(1, std::min<size_t>(8, kLdsBytes / tab_bytes)) : 8;
    const int64_t slots = (int64_t)device_cus() * blocks_per_cu;
    const int cpb_auto = (int)std::min<int64_t>(max_cpb, std::max<int64_t>(1, (n_chains + slots - 1) / slots));
    P->G = G;
    P->K = K;
    P->cpb = cpb_req > 0 ? std::min(cpb_req, max_cpb) : cpb_auto;
    P->lds = lds;
    P->tab_bytes = tab_bytes;
    P->tuned = false;
    P->tuned_ms = 0.0f;
    return NQS_OK;
}

nqs_status rbm_launch_plan(const RbmSampleArgs &A, const RbmPlan &P, bool trace, bool noise, int init,
                           hipStream_t stream)
{
    const int64_t blocks64 = (A.n_chains + P.cpb - 1) / P.cpb;
    if (blocks64 > INT32_MAX) return set_error(NQS_EINVAL, "too many chains");
    RbmLaunch L;
    L.K = P.K;
    L.threads = P.cpb * P.G;
    L.blocks = (int)blocks64;
    L.lds = P.lds;
    L.trace = trace;
    L.noise = noise;
    L.init = init;
    L.lds_bytes = P.lds ? P.tab_bytes : 0;
    switch (P.G) {
    case 16: return rbm_sample_launch_g16(A, L, stream);
    case 32: return rbm_sample_launch_g32(A, L, stream);
    default: return rbm_sample_launch_g64(A, L, stream);
    }
}

// The measured plan: every valid candidate among the lanes per chain `Gs`
// (all of 16, 32, 64 when Gs is NULL), both table placements and two
// chains-per-block counts is timed on a short burn-in from fresh start states
// of this model copy and chain count (scratch states, no outputs; the stream is
// synchronised), and the fastest is kept for the life of the process, keyed by
// (device, N, M, dtype, n_chains, candidate set).  Later calls reuse it, so
// results stay reproducible within a process.
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int64_t, int>, RbmPlan> g_tune;
}

nqs_status rbm_plan_tuned(nqs_model *m, const nqs_sample_cfg &cfg, const int *Gs, int nG, hipStream_t stream,
                          RbmPlan *out)
{
    static const int all[3] = {16, 32, 64};
    if (!Gs) {
        Gs = all;
        nG = 3;
    }
    nqs_status st = ensure_copy(m, cfg.dtype, stream);
    if (st != NQS_OK) return st;
    const RbmDev &net = m->copies[cfg.dtype].rbm;
    const int N = net.N, M = net.M;
    int dev = 0;
    NQS_HIP_TRY(hipGetDevice(&dev));
    int set = 0;
    for (int q = 0; q < nG; ++q) set |= Gs[q];
    const auto key = std::make_tuple(dev, N, M, (int)cfg.dtype, cfg.n_chains, set);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *out = it->second;
            return NQS_OK;
        }
    }
    std::vector<RbmPlan> cand;
    for (int q = 0; q < nG; ++q) {
        for (int lds = 1; lds >= 0; --lds) {
            RbmPlan P;
            if (rbm_plan_rule(N, M, cfg.n_chains, Gs[q], lds, 0, &P) != NQS_OK) continue;
            cand.push_back(P);
            if (P.cpb >= 2) {
                RbmPlan H;
                if (rbm_plan_rule(N, M, cfg.n_chains, Gs[q], lds, P.cpb / 2, &H) == NQS_OK) cand.push_back(H);
            }
        }
    }
    if (cand.empty()) return set_error(NQS_EUNSUPPORTED, "no lanes-per-chain candidate fits this RBM");
    const int64_t C = std::max<int64_t>(1, cfg.n_chains);
    const int64_t per_sweep = C * N;
    const int sweeps = (int)std::max<int64_t>(1, std::min<int64_t>(64, (4000000 + per_sweep - 1) / per_sweep));
    int8_t *scratch = nullptr;
    NQS_HIP_TRY(hipMalloc(&scratch, (size_t)C * N));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nqs_status result = NQS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventCreate failed");
    RbmSampleArgs A;
    std::memset(&A, 0, sizeof(A));
    A.net = net;
    A.chain_state = scratch;
    A.n_chains = C;
    A.n_sweeps = 0;
    A.n_burnin = sweeps;
    A.sweep_size = N;
    A.refresh_sweeps = cfg.refresh_sweeps > 0 ? cfg.refresh_sweeps : 1;
    A.seed = cfg.seed;
    A.inst = cfg.instance_id;
    RbmPlan best = cand[0];
    float best_ms = 3.4e38f;
    for (size_t q = 0; q < cand.size() && result == NQS_OK; ++q) {
        float t = 3.4e38f;
        for (int rep = 0; rep < 3 && result == NQS_OK; ++rep) {   // the first run warms up
            if (hipEventRecord(e0, stream) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventRecord failed");
            if (result == NQS_OK) result = rbm_launch_plan(A, cand[q], false, false, 1, stream);
            if (result == NQS_OK && hipEventRecord(e1, stream) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventRecord failed");
            if (result == NQS_OK && hipEventSynchronize(e1) != hipSuccess) result = set_error(NQS_EDEVICE, "tuning run failed");
            float ms = 0.0f;
            if (result == NQS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventElapsedTime failed");
            if (rep > 0) t = std::min(t, ms);
        }
        if (result == NQS_OK && t < best_ms) {
            best_ms = t;
            best = cand[q];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (result != NQS_OK) return result;
    best.tuned = true;
    best.tuned_ms = best_ms;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = best;
    }
    *out = best;
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// Local energies, TFIM:  eps(s) = J sum_<ij> s_i s_j + h sum_i psi(s^i)/psi(s),
// psi(s^i)/psi(s) = exp(-2 a_i s_i) prod_j (C_ij - s_i t_j S_ij),  t = tanh(W s + b).
// A block takes 16 samples.
//  Phase 1: theta = W s + b for the 16 samples on the matrix cores
//   (v_mfma_f32_16x16x4f32; hidden units x samples tiles spread over the waves),
//   t = tanh(theta) into LDS as tT[j][b] (row stride 20 floats).
//  Phase 2: Q adjacent lanes share a site i and split the hidden units
//   (lane q takes j = q, q + Q, ...), each keeping 16 running products; the
//   (C, S) pair is loaded once per (i, j) and used for 16 samples.  Products
//   are renormalised (frexp) every `renorm` factors, a count chosen on the host
//   from max |W| so that no partial product leaves the normal FP32 range.
//  Combine: a reduce-scatter butterfly over the Q lanes multiplies the partial
//   products and leaves 16/Q samples per lane; the per-site terms are formed in
//   FP32, converted, and summed over sites in FP64 in a fixed order.
// ---------------------------------------------------------------------------

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int Q, int B, bool RENORM>
__global__ void __launch_bounds__(1024) rbm_eloc_tfim_kernel(RbmDev net, const int8_t *__restrict__ samples,
                                                             int64_t n, int dim, int L, int pbc, double J, double h,
                                                             int renorm, double *__restrict__ eloc)
{
    constexpr int BL = B / Q;            // samples per lane after the butterfly
    constexpr int kElocTLd = B + 4;      // row stride of tT (floats)
    extern __shared__ __align__(16) float smem[];
    const int N = net.N, M = net.M;
    const int nwaves = blockDim.x >> 6;
    float *spT = smem;                                   // [N][B] spins as +-1
    float *tT = spT + (size_t)N * B;                     // [M][kElocTLd]
    double *red = (double *)(tT + (size_t)M * kElocTLd); // [nwaves][B]  (offset is a multiple of 16 floats)
    const int64_t base = (int64_t)blockIdx.x * B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int k = tid; k < N * B; k += blockDim.x) {
        const int b = k / N, i = k - b * N;
        const int64_t row = base + b;
        spT[i * B + b] = row < n ? (float)samples[row * N + i] : 1.0f;
    }
    __syncthreads();

    // phase 1: D[j][b] = sum_i W[j][i] s_i^b, 16 x 16 tiles; lane holds D[j0 + 4*(lane/16) + r][b0 + lane % 16].
    // W values of 8 contraction steps are loaded ahead of their matrix-core steps.
    {
        const int jt_count = (M + 15) >> 4, bt_count = (B + 15) >> 4, ksteps = (N + 3) >> 2;
        const int la = lane & 15, lk = lane >> 4;
        for (int t = wave; t < jt_count * bt_count; t += nwaves) {
            const int jt = t / bt_count, bt = t - (t / bt_count) * bt_count;
            const int j0 = jt * 16, ja = j0 + la, bc = bt * 16 + la;
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks0 = 0; ks0 < ksteps; ks0 += 8) {
                float av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = (ks0 + u) * 4 + lk;
                    const bool ok = ks0 + u < ksteps && k < N;
                    av[u] = (ok && ja < M) ? net.Wt[(size_t)k * M + ja] : 0.0f;
                    bv[u] = (ok && bc < B) ? spT[k * B + bc] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + 4 * lk + r;
                if (j < M && bc < B) tT[j * kElocTLd + bc] = tanhf(acc[r] + net.b[j]);
            }
        }
    }
    __syncthreads();

    // phase 2: lanes q of site i (item = i * Q + q)
    const int item = tid, i = item / Q, q = item - (item / Q) * Q;
    const bool active = i < N;
    float prod[B];
    int e2[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        prod[b] = 1.0f;
        e2[b] = 0;
    }
    if (active) {
        float si[B];
        const float4 *s4 = reinterpret_cast<const float4 *>(spT + i * B);
#pragma unroll
        for (int c = 0; c < B / 4; ++c) {
            const float4 v = s4[c];
            si[4 * c + 0] = v.x;
            si[4 * c + 1] = v.y;
            si[4 * c + 2] = v.z;
            si[4 * c + 3] = v.w;
        }
        const int iters = (M - q + Q - 1) / Q;
        // (C, S) of hidden unit j = t Q + q; the load for the next unit is issued one step
        // ahead (CSt carries 8 N slack entries, so the step past the last unit stays inside)
        const size_t cstep = (size_t)Q * N;
        const float2 *csp = net.CSt + (size_t)q * N + i;
        const float *tp = tT + q * kElocTLd;
        float2 cs = *csp;
        int t = 0;
        while (t < iters) {
            const int t1 = RENORM ? min(iters, t + renorm) : iters;
            for (; t < t1; ++t) {
                csp += cstep;
                const float2 nxt = *csp;
                const float4 *t4 = reinterpret_cast<const float4 *>(tp);
                tp += Q * kElocTLd;
#pragma unroll
                for (int c = 0; c < B / 4; ++c) {
                    const float4 tv = t4[c];
                    prod[4 * c + 0] *= fmaf(-tv.x * si[4 * c + 0], cs.y, cs.x);
                    prod[4 * c + 1] *= fmaf(-tv.y * si[4 * c + 1], cs.y, cs.x);
                    prod[4 * c + 2] *= fmaf(-tv.z * si[4 * c + 2], cs.y, cs.x);
                    prod[4 * c + 3] *= fmaf(-tv.w * si[4 * c + 3], cs.y, cs.x);
                }
                cs = nxt;
            }
#pragma unroll
            for (int b = 0; b < B; ++b) {
                int e;
                prod[b] = frexpf(prod[b], &e);
                e2[b] += e;
            }
        }
    }
    // reduce-scatter over the Q lanes: after the step with bit m, a lane keeps
    // the upper or lower half of its samples according to bit m of q
    int keep_base = 0;   // first sample index held (in units of the full B)
#pragma unroll
    for (int step = 0, half = B / 2; half >= BL; ++step, half >>= 1) {
        const int bit = (q >> step) & 1;
#pragma unroll
        for (int b = 0; b < half; ++b) {
            const float pk = bit ? prod[b + half] : prod[b], ps = bit ? prod[b] : prod[b + half];
            const int ek = bit ? e2[b + half] : e2[b], es = bit ? e2[b] : e2[b + half];
            const float pr = __shfl_xor(ps, 1 << step, 64);
            const int er = __shfl_xor(es, 1 << step, 64);
            int e;
            prod[b] = frexpf(pk * pr, &e);
            e2[b] = ek + er + e;
        }
        keep_base += bit * half;
    }
    // this lane now holds samples keep_base .. keep_base + BL - 1 of site i
    double contrib[BL];
#pragma unroll
    for (int b = 0; b < BL; ++b) contrib[b] = 0.0;
    if (active) {
        int nb1 = -1, nb2 = -1;
        if (dim == 1) {
            if (i + 1 < L) nb1 = i + 1;
            else if (pbc) nb1 = 0;
        } else {
            const int x = i / L, y = i - (i / L) * L;
            if (x + 1 < L) nb1 = (x + 1) * L + y;
            else if (pbc) nb1 = y;
            if (y + 1 < L) nb2 = x * L + y + 1;
            else if (pbc) nb2 = x * L;
        }
        const float ai = net.a[i];
#pragma unroll
        for (int b = 0; b < BL; ++b) {
            const int bb = keep_base + b;
            const float s = spT[i * B + bb];
            const float ratio = ldexpf(__expf(-2.0f * ai * s) * prod[b], e2[b]);
            float zz = 0.0f;
            if (nb1 >= 0) zz += spT[nb1 * B + bb];
            if (nb2 >= 0) zz += spT[nb2 * B + bb];
            contrib[b] = J * (double)(s * zz) + h * (double)ratio;
        }
    }
    // sum over the sites of the wave: lanes with equal q hold the same samples
#pragma unroll
    for (int off = Q; off < 64; off <<= 1)
#pragma unroll
        for (int b = 0; b < BL; ++b) contrib[b] += __shfl_xor(contrib[b], off, 64);
    if (lane < Q) {
#pragma unroll
        for (int b = 0; b < BL; ++b) red[wave * B + keep_base + b] = contrib[b];
    }
    __syncthreads();
    if (tid < B) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[w * B + tid];
        const int64_t row = base + tid;
        if (row < n) eloc[row] = s;
    }
}

template <int Q, int B, bool RENORM>
static nqs_status launch_eloc_q(const RbmDev &net, const nqs_ham_desc &ham, const int8_t *samples, int64_t n,
                                int renorm, double *eloc, hipStream_t stream)
{
    const int N = net.N, M = net.M;
    const int threads = std::max(64, (int)(((int64_t)N * Q + 63) / 64 * 64));
    const size_t lds = sizeof(float) * ((size_t)N * B + (size_t)M * (B + 4)) + sizeof(double) * (threads / 64) * B;
    if (lds > kLdsBytes) return set_error(NQS_EUNSUPPORTED, "RBM too large for the local-energy kernel");
    const int64_t blocks = (n + B - 1) / B;
    if (blocks > INT32_MAX) return set_error(NQS_EINVAL, "too many samples");
    allow_lds(rbm_eloc_tfim_kernel<Q, B, RENORM>, lds);
    hipLaunchKernelGGL((rbm_eloc_tfim_kernel<Q, B, RENORM>), dim3((unsigned)blocks), dim3(threads), lds, stream, net, samples,
                       n, ham.dim, ham.L, ham.pbc, ham.J, ham.h, renorm, eloc);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status rbm_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                            double *eloc, hipStream_t stream)
{
    if (ham.kind != NQS_TFIM)
        return set_error(NQS_EUNSUPPORTED, "RBM local energies are implemented for the TFIM");
    nqs_status st = ensure_copy(m, dtype, stream);
    if (st != NQS_OK) return st;
    const RbmDev &net = m->copies[dtype].rbm;
    if (!(net.max_abs_w <= kMaxAbsW)) return set_error(NQS_EUNSUPPORTED, "product-form ratios need |W| <= 5");
    const int N = net.N, M = net.M;
    if (N > 1024) return set_error(NQS_EUNSUPPORTED, "RBM local energies need N <= 1024");
    // two lanes per site (measured best on the 10x10 lattice against 1, 4 and 8), one when
    // 2N lanes do not fit in a block; 16 samples per block (32 costs occupancy)
    const int Q = (2 * N <= 1024 && M >= 2) ? 2 : 1;
    // factors lie in [e^{-2|W|}, e^{2|W|}]: a run of k of them after a renormalisation
    // stays within 2^{+-120} when k * 2|W| / ln 2 <= 119
    const double per = 2.0 * (double)net.max_abs_w / 0.6931471805599453;
    const int iters = (M + Q - 1) / Q;
    int renorm = per > 0.0 ? (int)std::min<double>((double)iters, std::floor(119.0 / per)) : iters;
    renorm = std::max(1, renorm);
    const bool rn = renorm < iters;
    constexpr int B = 16;
#define NQS_ELOC_CASE(QQ, BB)                                                                          \
    if (Q == QQ && B == BB)                                                                            \
        return rn ? launch_eloc_q<QQ, BB, true>(net, ham, samples, n, renorm, eloc, stream)            \
                  : launch_eloc_q<QQ, BB, false>(net, ham, samples, n, renorm, eloc, stream);
    NQS_ELOC_CASE(2, 16)
    NQS_ELOC_CASE(1, 16)
#undef NQS_ELOC_CASE
    return set_error(NQS_EDEVICE, "no local-energy kernel for this shape");
}

// ---------------------------------------------------------------------------
// log psi and O_k: O_a = s, O_b = tanh theta, O_W[j][i] = tanh(theta_j) s_i.
// B samples per block; the O rows are written with consecutive threads on
// consecutive parameters (HBM-write bound).
// ---------------------------------------------------------------------------
template <int B>
__global__ void __launch_bounds__(256) rbm_grad_kernel(RbmDev net, const int8_t *__restrict__ samples, int64_t n,
                                                       float *__restrict__ logpsi, float *__restrict__ O,
                                                       float *__restrict__ Tout, int64_t p0, int64_t p1)
{
    extern __shared__ float smem[];
    const int N = net.N, M = net.M;
    float *spT = smem;                   // [N][B]
    float *tT = spT + (size_t)N * B;     // [M][B]
    float *red = tT + (size_t)M * B;     // [nwaves][B]
    const int64_t base = (int64_t)blockIdx.x * B;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;

    for (int k = tid; k < N * B; k += nt) {
        const int b = k / N, i = k - b * N;
        const int64_t row = base + b;
        spT[i * B + b] = row < n ? (float)samples[row * N + i] : 1.0f;
    }
    __syncthreads();
    float part[B];
#pragma unroll
    for (int b = 0; b < B; ++b) part[b] = 0.0f;
    for (int j = tid; j < M; j += nt) {
        float th[B];
#pragma unroll
        for (int b = 0; b < B; ++b) th[b] = net.b[j];
        for (int i = 0; i < N; ++i) {
            const float w = net.Wt[(size_t)i * M + j];
#pragma unroll
            for (int b = 0; b < B; ++b) th[b] = fmaf(w, spT[i * B + b], th[b]);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const float t = tanhf(th[b]);
            tT[j * B + b] = t;
            part[b] += logcosh_f32(th[b]);
            if (Tout && base + b < n) Tout[(base + b) * M + j] = t;
        }
    }
    for (int i = tid; i < N; i += nt) {
#pragma unroll
        for (int b = 0; b < B; ++b) part[b] = fmaf(net.a[i], spT[i * B + b], part[b]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float v = group_sum<64>(part[b]);
        if (lane == 0) red[wv * B + b] = v;
    }
    __syncthreads();
    if (logpsi && tid < B && base + tid < n) {
        float s = 0.0f;
        for (int w = 0; w < nw; ++w) s += red[w * B + tid];
        logpsi[base + tid] = s;
    }
    if (!O) return;
    // columns [p0, p1) of the parameter order (a, b, W), row stride p1 - p0
    const int64_t NM = (int64_t)N + M, ldo = p1 - p0;
    const int64_t q0 = max(p0 - NM, (int64_t)0), q1 = min(p1 - NM, (int64_t)M * N);
    for (int b = 0; b < B; ++b) {
        const int64_t row = base + b;
        if (row >= n) break;
        float *o = O + row * ldo - p0;   // o[p] for p in [p0, p1)
        for (int64_t p = p0 + tid; p < min(p1, NM); p += nt) o[p] = p < N ? spT[p * B + b] : tT[(p - N) * B + b];
        // W block: q = j*N + i, advanced by nt per iteration with (j, i) carried
        int j = (int)((q0 + tid) / N), i = (int)((q0 + tid) - (int64_t)j * N);
        const int dj = nt / N, di = nt - (nt / N) * N;
        float *ow = o + NM;
        for (int64_t q = q0 + tid; q < q1; q += nt) {
            ow[q] = tT[j * B + b] * spT[i * B + b];
            i += di;
            j += dj;
            if (i >= N) {
                i -= N;
                ++j;
            }
        }
    }
}

// vjp_out[p] = sum_k g_k O[k][p] using the per-sample tanh values T[n][M].
__global__ void rbm_vjp_kernel(int N, int M, const int8_t *__restrict__ samples, const float *__restrict__ T,
                               const float *__restrict__ g, int64_t n, float *__restrict__ out)
{
    const int64_t P = (int64_t)N + M + (int64_t)M * N;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        if (p < N) {
            for (int64_t k = 0; k < n; ++k) acc += (double)g[k] * samples[k * N + p];
        } else if (p < N + M) {
            const int j = (int)(p - N);
            for (int64_t k = 0; k < n; ++k) acc += (double)g[k] * T[k * M + j];
        } else {
            const int64_t q = p - N - M;
            const int j = (int)(q / N), i = (int)(q - (q / N) * N);
            for (int64_t k = 0; k < n; ++k) acc += (double)g[k] * T[k * M + j] * samples[k * N + i];
        }
        out[p] = (float)acc;
    }
}

nqs_status rbm_tanh_theta(nqs_model *m, const int8_t *samples, int64_t n, float *t, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const RbmDev &net = m->copies[NQS_F32].rbm;
    constexpr int B = 8;
    const int threads = 256;
    const size_t lds = sizeof(float) * ((size_t)net.N * B + (size_t)net.M * B + (threads / 64) * B);
    if (lds > kLdsBytes) return set_error(NQS_EUNSUPPORTED, "RBM too large for the gradient kernel");
    const int64_t blocks = (n + B - 1) / B;
    if (blocks > INT32_MAX) return set_error(NQS_EINVAL, "too many samples");
    allow_lds(rbm_grad_kernel<B>, lds);
    hipLaunchKernelGGL((rbm_grad_kernel<B>), dim3((unsigned)blocks), dim3(threads), lds, stream, net, samples, n,
                       nullptr, nullptr, t, (int64_t)0, (int64_t)0);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status rbm_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                           const float *vjp_in, float *vjp_out, hipStream_t stream, int64_t p0, int64_t p1)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const RbmDev &net = m->copies[NQS_F32].rbm;
    const int N = net.N, M = net.M;
    constexpr int B = 8;
    const int threads = 256;
    const size_t lds = sizeof(float) * ((size_t)N * B + (size_t)M * B + (threads / 64) * B);
    if (lds > kLdsBytes) return set_error(NQS_EUNSUPPORTED, "RBM too large for the gradient kernel");
    float *T = nullptr;
    if (vjp_in) {
        T = (float *)workspace(sizeof(float) * (size_t)n * M, stream);
        if (!T) return set_error(NQS_ENOMEM, "workspace allocation failed");
    }
    const int64_t blocks = (n + B - 1) / B;
    if (blocks > INT32_MAX) return set_error(NQS_EINVAL, "too many samples");
    if (logpsi || O || T) {
        allow_lds(rbm_grad_kernel<B>, lds);
        hipLaunchKernelGGL((rbm_grad_kernel<B>), dim3((unsigned)blocks), dim3(threads), lds, stream, net, samples, n,
                           logpsi, O, T, p0, p1);
        NQS_HIP_TRY(hipGetLastError());
    }
    if (vjp_in) {
        const int64_t P = m->P;
        const int vb = (int)std::min<int64_t>((P + 255) / 256, 65535);
        hipLaunchKernelGGL(rbm_vjp_kernel, dim3(vb), dim3(256), 0, stream, N, M, samples, T, vjp_in, n, vjp_out);
        NQS_HIP_TRY(hipGetLastError());
    }
    return NQS_OK;
}

}  // namespace nqs
