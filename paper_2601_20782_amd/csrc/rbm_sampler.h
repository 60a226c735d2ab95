// RBM single-flip Metropolis-Hastings sampler (App. G network, Sec. III.A
// acceptance, App. C single-bit-flip proposal), instantiated per lanes-per-chain G.
//
// One chain per group of G lanes; lane g of the group owns hidden units
// j = g, g+G, ..., g+(K-1)G and spin word g (32 spins per word).  Per hidden
// unit the chain keeps (c_j, s_j) proportional to (cosh theta_j, sinh theta_j),
// theta = W s + b, with the common factor reset to 1 at each refresh, and per
// lane the running log2 of its c_j product.  Flipping site i moves theta_j to
// theta_j - 2 s_i W_ji; with C = cosh 2W_ji, S = sinh 2W_ji the cosh and sinh
// addition formulas give
//   n_j = c_j C - s_i s_j S  = c_j cosh(theta_j - 2 s_i W_ji) / cosh(theta_j),
//   log2 |psi(s')/psi(s)|^2 = -4 a_i s_i / ln 2 + 2 sum_j [log2 n_j - log2 c_j],
// and an accepted flip sets c_j <- n_j, s_j <- s_j C - s_i c_j S.  The move is
// accepted iff log2 u < that log-ratio, i.e. u < min(1, |psi(s')/psi(s)|^2).
// The (C,S) table (plus one neutral entry (1,0) used by lanes past the last
// hidden unit) lives in LDS when it fits, else it is read through L2; the
// table column of the next proposal is loaded while the current one is
// decided.  Group sums use DPP and end in one lane, read back with
// v_readlane, so every lane of a chain takes the same decision.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace nqs {

constexpr float kLn2 = 0.69314718055994531f;

// tanh from one exponential: tanh|x| = (1 - e^{-2|x|}) / (1 + e^{-2|x|})
__device__ __forceinline__ float tanh_fast(float x)
{
    const float e = __expf(-2.0f * fabsf(x));
    return copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), x);
}

// theta = W s + b from scratch: c = 1, s = tanh theta; returns log psi (FP32)
// when want_f, else 0.
template <int G, int K>
__device__ __forceinline__ float rbm_refresh(const RbmDev &net, uint32_t word, int gl, float (&c)[K], float (&sh)[K],
                                             float &lpart, bool want_f = true)
{
    const int N = net.N, M = net.M;
    constexpr int CH = K >= 8 ? 2 : (K >= 4 ? 4 : 8);   // sites whose W rows are in flight together
    float th[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = gl + k * G;
        th[k] = j < M ? net.b[j] : 0.0f;
    }
    const int jl = gl + (K - 1) * G;
    const int jlast = jl < M ? jl : M - 1;          // clamp the tail slot to a valid column
    const float wlast = jl < M ? 1.0f : 0.0f;
    float as = 0.0f;
    const int NW = (N + 31) >> 5;
    for (int w = 0; w < NW; ++w) {
        const uint32_t bits = group_bcast<G>(word, w);
        const int i0 = w << 5;
        const int nb = min(32, N - i0);
        int bb = 0;
        for (; bb + CH <= nb; bb += CH) {
            float wv[CH][K];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const float *wrow = net.Wt + (size_t)(i0 + bb + q) * M + gl;
#pragma unroll
                for (int k = 0; k < K - 1; ++k) wv[q][k] = wrow[k * G];
                wv[q][K - 1] = net.Wt[(size_t)(i0 + bb + q) * M + jlast];
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const float s = ((bits >> (bb + q)) & 1u) ? 1.0f : -1.0f;
                as = fmaf(net.a[i0 + bb + q], s, as);
#pragma unroll
                for (int k = 0; k < K - 1; ++k) th[k] = fmaf(wv[q][k], s, th[k]);
                th[K - 1] = fmaf(wv[q][K - 1] * wlast, s, th[K - 1]);
            }
        }
        for (; bb < nb; ++bb) {
            const int i = i0 + bb;
            const float s = ((bits >> bb) & 1u) ? 1.0f : -1.0f;
            as = fmaf(net.a[i], s, as);
            const float *wrow = net.Wt + (size_t)i * M + gl;
#pragma unroll
            for (int k = 0; k < K - 1; ++k) th[k] = fmaf(wrow[k * G], s, th[k]);
            th[K - 1] = fmaf(net.Wt[(size_t)i * M + jlast] * wlast, s, th[K - 1]);
        }
    }
    lpart = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        c[k] = 1.0f;
        const bool valid = (k < K - 1) || (jl < M);
        sh[k] = valid ? tanh_fast(th[k]) : 0.0f;
    }
    if (!want_f) return 0.0f;
    float lc = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool valid = (k < K - 1) || (jl < M);
        lc += valid ? logcosh_f32(th[k]) : 0.0f;
    }
    return as + group_sum_uniform<G>(lc);
}

// Proposals of one batch: lane g of a group holds site, log2 u, u bits and the
// bias term of proposal (batch start + g).
struct PropBatch {
    uint32_t i, ub;
    float l2u, a2;
};

__device__ __forceinline__ PropBatch make_batch(const RbmDev &net, uint64_t step, uint32_t gid, uint32_t inst,
                                                uint32_t key0, uint32_t key1)
{
    const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, inst << 8, key0, key1);
    PropBatch pb;
    pb.i = (uint32_t)index_from_word(rb.r0, net.N);
    pb.ub = rb.r2 >> 8;
    pb.l2u = __builtin_amdgcn_logf((float)pb.ub * 5.9604644775390625e-8f);   // log2(u), u = ub * 2^-24
    pb.a2 = net.a2[pb.i];
    return pb;
}

template <int G, int K, bool LDS_TAB>
__device__ __forceinline__ void load_column(const float2 *__restrict__ tab, int i, int M, int gl, int last_off,
                                            bool last_ok, float2 (&cs)[K])
{
    const int base = i * M + gl;
#pragma unroll
    for (int k = 0; k < K - 1; ++k) cs[k] = tab[base + k * G];
    cs[K - 1] = tab[last_ok ? base + (K - 1) * G : last_off];
}

// zeta(x) / ln 2 of the noisy target, log pi~ = log pi + zeta: Philox4x32-10 with
// the configuration's four 32-bit words as the counter (spin i up = bit i % 32 of
// word i / 32) and the noise seed as the key, then Box-Muller on the first two
// outputs, u1 in (0, 1] and u2 in [0, 1) on the 2^-24 grid.
__device__ __forceinline__ float noise_zeta_log2(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                                 const RbmSampleArgs &A)
{
    const Block4 r = philox4x32_10(w0, w1, w2, w3, A.noise_key0, A.noise_key1);
    const float u1 = (float)((r.r0 >> 8) + 1u) * 5.9604644775390625e-8f;
    const float u2 = (float)(r.r1 >> 8) * 5.9604644775390625e-8f;
    const float g = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
    return A.noise_sigma * g * 1.4426950408889634f;
}

// Runs chain c on the G lanes of its group (gl = lane in group).  s_tab is the
// LDS copy of the table when LDS_TAB.  With init, the start state is drawn
// from the init stream (counter tag 1, spin i = bit i%32 of word i/32) instead
// of being read from chain_state.
// With NOISE the target is the noisy pi~ (every lane keeps all configuration words).
template <int G, int K, bool LDS_TAB, bool TRACE, bool NOISE = false>
__device__ __forceinline__ void rbm_run_chain(const RbmSampleArgs &A, int64_t c, int gl, const float2 *s_tab, bool init)
{
    const int N = A.net.N, M = A.net.M;
    const float2 *tab = A.net.CS;
    const uint32_t gid = A.chain_id_offset + (uint32_t)c;
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    const int NW = (N + 31) >> 5;
    const int last_off = N * M;
    const bool last_ok = gl + (K - 1) * G < M;

    uint32_t word = 0;
    if (gl < NW) {
        const int nb = min(32, N - gl * 32);
        if (init) {
            const Block4 ib = stream_block(A.seed, (uint64_t)(gl >> 2), gid, A.inst, 1u);
            const uint32_t r = (gl & 3) == 0 ? ib.r0 : (gl & 3) == 1 ? ib.r1 : (gl & 3) == 2 ? ib.r2 : ib.r3;
            word = nb == 32 ? r : (r & ((1u << nb) - 1u));
        } else {
            const int8_t *src = A.chain_state + (size_t)c * N + gl * 32;
            for (int bb = 0; bb < nb; ++bb) word |= (src[bb] > 0 ? 1u : 0u) << bb;
        }
    }

    float cc[K], sh[K], lpart;
    const bool diag = TRACE && A.dg_drift != nullptr;
    float f = rbm_refresh<G, K>(A.net, word, gl, cc, sh, lpart, diag);
    unsigned long long dg_nonfinite = 0, dg_acc0 = 0;
    uint32_t dg_run = 0, dg_longest = 0;
    float dg_f = f, dg_drift = 0.0f;   // log psi carried by the accepted log-ratios since the last refresh
    uint32_t nw0 = 0u, nw1 = 0u, nw2 = 0u, nw3 = 0u;
    float zc = 0.0f;
    if constexpr (NOISE) {
        nw0 = group_bcast<G>(word, 0);
        if (NW > 1) nw1 = group_bcast<G>(word, 1);
        if (NW > 2) nw2 = group_bcast<G>(word, 2);
        if (NW > 3) nw3 = group_bcast<G>(word, 3);
        zc = noise_zeta_log2(nw0, nw1, nw2, nw3, A);
    }

    const int sw = A.sweep_size;
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * sw;
    unsigned long long acc = 0;
    int in_sweep = 0;
    int since_refresh = 0;
    int64_t sweep = 0;
    const bool want_out = (A.samples != nullptr) || (A.logpsi != nullptr);

    // proposal pipeline: `cur` covers steps [base, base+G), `nxt` the next G
    uint64_t base = A.step_offset;
    PropBatch cur = make_batch(A.net, base + gl, gid, A.inst, key0, key1);
    PropBatch nxt = make_batch(A.net, base + G + gl, gid, A.inst, key0, key1);
    int p = 0;
    int i_c = (int)group_bcast<G>(cur.i, 0);
    uint32_t ub_c = group_bcast<G>(cur.ub, 0);
    float l2u_c = __uint_as_float(group_bcast<G>(__float_as_uint(cur.l2u), 0));
    float a2_c = __uint_as_float(group_bcast<G>(__float_as_uint(cur.a2), 0));
    float2 csA[K], csB[K];
    if constexpr (LDS_TAB) load_column<G, K, true>(s_tab, i_c, M, gl, last_off, last_ok, csA);
    else load_column<G, K, false>(tab, i_c, M, gl, last_off, last_ok, csA);

    // one proposal: evaluate with cs_c (column of i_c), prefetch the next column into cs_n
    auto step = [&](int64_t k, float2 (&cs_c)[K], float2 (&cs_n)[K]) {
        const int pn = p + 1;
        int i_n;
        uint32_t ub_n;
        float l2u_n, a2_n;
        if (pn < G) {
            i_n = (int)group_bcast<G>(cur.i, pn);
            ub_n = group_bcast<G>(cur.ub, pn);
            l2u_n = __uint_as_float(group_bcast<G>(__float_as_uint(cur.l2u), pn));
            a2_n = __uint_as_float(group_bcast<G>(__float_as_uint(cur.a2), pn));
        } else {
            i_n = (int)group_bcast<G>(nxt.i, 0);
            ub_n = group_bcast<G>(nxt.ub, 0);
            l2u_n = __uint_as_float(group_bcast<G>(__float_as_uint(nxt.l2u), 0));
            a2_n = __uint_as_float(group_bcast<G>(__float_as_uint(nxt.a2), 0));
        }
        if constexpr (LDS_TAB) load_column<G, K, true>(s_tab, i_n, M, gl, last_off, last_ok, cs_n);
        else load_column<G, K, false>(tab, i_n, M, gl, last_off, last_ok, cs_n);

        // proposal k: flip site i_c;  S' = s_i S by flipping the sign bit
        const uint32_t wbits = group_bcast<G>(word, i_c >> 5);
        const bool up = (wbits >> (i_c & 31)) & 1u;
        const uint32_t smask = up ? 0u : 0x80000000u;
        float sp[K], nn[K];
        float prod = 1.0f;
        int e2 = 0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            sp[q] = __uint_as_float(__float_as_uint(cs_c[q].y) ^ smask);
            nn[q] = fmaf(-sh[q], sp[q], cc[q] * cs_c[q].x);
            prod *= nn[q];
            if ((q & 7) == 7 && q + 1 < K) {
                int e;
                prod = frexpf(prod, &e);
                e2 += e;
            }
        }
        const float lnew = __builtin_amdgcn_logf(prod) + (float)e2;    // log2
        const float dsum = group_sum_uniform<G>(lnew - lpart);
        float d2 = fmaf(2.0f, dsum, up ? -a2_c : a2_c);                // log2 of the acceptance ratio
        float zn = 0.0f;
        const uint32_t fbit = 1u << (i_c & 31);
        const int fw = i_c >> 5;
        if constexpr (NOISE) {
            zn = noise_zeta_log2(nw0 ^ (fw == 0 ? fbit : 0u), nw1 ^ (fw == 1 ? fbit : 0u),
                                 nw2 ^ (fw == 2 ? fbit : 0u), nw3 ^ (fw == 3 ? fbit : 0u), A);
            d2 += zn - zc;
        }
        const bool accept = l2u_c < d2;                                // NaN rejects
        if (accept) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                sh[q] = fmaf(-cc[q], sp[q], sh[q] * cs_c[q].x);
                cc[q] = nn[q];
            }
            lpart = lnew;
            if (gl == (i_c >> 5)) word ^= 1u << (i_c & 31);
            if constexpr (NOISE) {
                nw0 ^= fw == 0 ? fbit : 0u;
                nw1 ^= fw == 1 ? fbit : 0u;
                nw2 ^= fw == 2 ? fbit : 0u;
                nw3 ^= fw == 3 ? fbit : 0u;
                zc = zn;
            }
            ++acc;
        }
        if constexpr (TRACE) {
            if (diag) {
                dg_nonfinite += __builtin_isfinite(d2) ? 0ull : 1ull;
                if (accept) dg_f = fmaf(d2, 0.5f * kLn2, dg_f);
            }
            if (c < A.n_traced && gl == 0) {
                const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                A.tr_site[idx] = i_c | (0xFFFF << 16);
                A.tr_ubits[idx] = ub_c;
                A.tr_delta[idx] = d2 * kLn2;
                A.tr_acc[idx] = accept ? 1 : 0;
            }
        }
        // advance the pipeline
        i_c = i_n;
        ub_c = ub_n;
        l2u_c = l2u_n;
        a2_c = a2_n;
        p = pn;
        if (p == G) {
            p = 0;
            base += G;
            cur = nxt;
            nxt = make_batch(A.net, base + G + gl, gid, A.inst, key0, key1);
        }
        if (++in_sweep == sw) {
            in_sweep = 0;
            const int64_t out = sweep - A.n_burnin;
            const bool emit = want_out && out >= 0;
            const bool need_logpsi = A.logpsi != nullptr && out >= 0;
            if constexpr (TRACE) {
                if (diag) {
                    dg_run = acc == dg_acc0 ? dg_run + 1 : 0;
                    dg_longest = max(dg_longest, dg_run);
                    dg_acc0 = acc;
                }
            }
            if (++since_refresh == A.refresh_sweeps || need_logpsi) {
                f = rbm_refresh<G, K>(A.net, word, gl, cc, sh, lpart, need_logpsi || diag);
                since_refresh = 0;
                if constexpr (TRACE) {
                    if (diag) {
                        dg_drift = fmaxf(dg_drift, fabsf(dg_f - f));
                        dg_f = f;
                    }
                }
            }
            if (emit) {
                if (A.samples && gl < NW) {
                    int8_t *dst = A.samples + ((size_t)out * A.n_chains + c) * N + gl * 32;
                    const int nb = min(32, N - gl * 32);
                    for (int bb = 0; bb < nb; ++bb) dst[bb] = ((word >> bb) & 1u) ? 1 : -1;
                }
                if (A.logpsi && gl == 0) A.logpsi[(size_t)out * A.n_chains + c] = f;
            }
            ++sweep;
        }
    };

    int64_t k = 0;
    for (; k + 1 < total; k += 2) {
        step(k, csA, csB);
        step(k + 1, csB, csA);
    }
    if (k < total) step(k, csA, csB);

    if (gl < NW) {
        int8_t *dst = A.chain_state + (size_t)c * N + gl * 32;
        const int nb = min(32, N - gl * 32);
        for (int bb = 0; bb < nb; ++bb) dst[bb] = ((word >> bb) & 1u) ? 1 : -1;
    }
    if (A.n_acc && gl == 0) A.n_acc[c] = acc;
    if constexpr (TRACE) {
        if (diag && gl == 0) {
            A.dg_nonfinite[c] = dg_nonfinite;
            A.dg_stuck[c] = dg_longest;
            A.dg_drift[c] = dg_drift;
        }
    }
}

template <int G, int K, bool LDS_TAB, bool TRACE, bool NOISE = false>
__global__ void __launch_bounds__(G == 16 ? 256 : (G == 32 ? 512 : 1024)) rbm_sample_kernel(RbmSampleArgs A, int init)
{
    extern __shared__ float2 s_tab[];
    const int N = A.net.N, M = A.net.M;
    if constexpr (LDS_TAB) {
        const int total = N * M + 1;   // includes the neutral entry
        for (int k = threadIdx.x; k < total; k += blockDim.x) s_tab[k] = A.net.CS[k];
        __syncthreads();
    }
    const int cpb = blockDim.x / G;
    const int gl = threadIdx.x % G;
    const int64_t c = (int64_t)blockIdx.x * cpb + threadIdx.x / G;
    if (c >= A.n_chains) return;   // whole groups leave together; no barrier follows
    rbm_run_chain<G, K, LDS_TAB, TRACE, NOISE>(A, c, gl, s_tab, init != 0);
}

template <int G, int K>
static void launch_rbm_sample_gk(const RbmSampleArgs &A, const RbmLaunch &L, hipStream_t s)
{
    if (L.noise) {   // table in LDS, no trace (checked by the launcher)
        allow_lds(rbm_sample_kernel<G, K, true, false, true>, L.lds_bytes);
        hipLaunchKernelGGL((rbm_sample_kernel<G, K, true, false, true>), dim3(L.blocks), dim3(L.threads), L.lds_bytes, s,
                           A, L.init);
        return;
    }
    if (L.lds) {
        if (L.trace) {
            allow_lds(rbm_sample_kernel<G, K, true, true>, L.lds_bytes);
            hipLaunchKernelGGL((rbm_sample_kernel<G, K, true, true>), dim3(L.blocks), dim3(L.threads), L.lds_bytes, s, A, L.init);
        } else {
            allow_lds(rbm_sample_kernel<G, K, true, false>, L.lds_bytes);
            hipLaunchKernelGGL((rbm_sample_kernel<G, K, true, false>), dim3(L.blocks), dim3(L.threads), L.lds_bytes, s, A, L.init);
        }
    } else {
        if (L.trace) hipLaunchKernelGGL((rbm_sample_kernel<G, K, false, true>), dim3(L.blocks), dim3(L.threads), 0, s, A, L.init);
        else hipLaunchKernelGGL((rbm_sample_kernel<G, K, false, false>), dim3(L.blocks), dim3(L.threads), 0, s, A, L.init);
    }
}

}  // namespace nqs
