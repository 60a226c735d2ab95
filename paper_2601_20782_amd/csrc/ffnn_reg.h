// Two-layer dense network with layer 2 held in registers (16-bit operands).
//   z1 = W1 s + b1,  h1 = ReLU(z1),  z2 = W2 h1 + b2,  log|psi| = sum_k log cosh(z2_k).
//
// A block of 512 threads (8 waves) keeps W2 resident for its whole life: wave w
// holds output rows 32w .. 32w+31 of W2 as the A fragments of
// v_mfma_f32_32x32x16_{bf16,f16} (KE = ceil(m1 / 16) fragments of 8 values per
// lane, K = 16 per fragment; W2's padding columns past m1 are never multiplied).  The rows to evaluate are staged once per pass into LDS as the B
// operand (h1 rows, one row per matrix column), so the only per-pass traffic is
// LDS reads of h1; no weight is re-read from L2 inside the loop.  Each wave
// turns its 32 x 32 tile into per-row partial log-cosh sums over its 32
// outputs; the partials of the waves are added in wave order.
//
// Sampler: 64 chains per block; wave w keeps z1 of chains 8w .. 8w+7 in
// registers (lane c owns hidden units 8c .. 8c + 7, so that a W1 column or an h1
// row moves in one 16-byte access per lane) and updates it by the rank-1
// (flip) or rank-2 (exchange) change of an accepted move.  Proposals that
// change nothing (an exchange of equal spins) are compacted away before the
// matrix product, so a pass evaluates only the effective proposals.
// Local energies: groups of samples whose connected configurations are listed,
// laid end to end and evaluated 32 rows per pass, W1 and the rows in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "ffnn_mc.h"

namespace nqs {

constexpr int kRegThreads = 512;
constexpr int kRegWaves = kRegThreads / 64;
constexpr int kRegRows = 64;       // chains per sampler block

// A fragments of this wave's 32 rows of W2 ([m2p][m1p], operand format); zero
// beyond m2p.
template <typename T, int KF>
__device__ __forceinline__ void reg_load_w2(const T *__restrict__ W2, int m1p, int m2p,
                                            typename Mc<T>::frag (&a)[KF])
{
    typedef typename Mc<T>::frag frag;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int out = wave * 32 + (lane & 31);
    const int kofs = 8 * (lane >> 5);
#pragma unroll
    for (int kf = 0; kf < KF; ++kf) {
        if (out < m2p) {
            a[kf] = *reinterpret_cast<const frag *>(W2 + (size_t)out * m1p + kf * 16 + kofs);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) a[kf][e] = Mc<T>::from_f32(0.0f);
        }
    }
}

// Four of the 16 outputs a lane holds of a 32 x 32 tile (registers 4q .. 4q + 3: outputs
// 8q + 4 (lane / 32) + 0..3 of the wave's 32) into the running |z| sum and product of (1 + e^-2|z|).
__device__ __forceinline__ void eloc_logcosh4(const mc_floatx16 &acc, int q, float4 b, float &abs_sum, float &prod)
{
    const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float v = fabsf(acc[4 * q + r] + bb[r]);
        abs_sum += v;
        prod = fmaf(prod, __builtin_amdgcn_exp2f(v * -2.8853900817779268f), prod);   // e^-2v = 2^(-2 log2(e) v)
    }
}

// Rows row0 .. row0+31 of Hs (ldh elements per row) through layer 2 and the
// log-cosh sum over this wave's 32 outputs; lanes 0..31 return the partial of
// row row0 + lane (lanes 32..63 the same value).  Each B fragment is read two
// products ahead of its use, the order pinned against the scheduler.  Outputs
// past m2 have zero W2 rows and a zero bias, so z2 = 0 exactly and they add
// log cosh 0 = 0 (the caller skips waves with no real output).
template <typename T, int KF>
__device__ __forceinline__ float reg_tile_logcosh(const typename Mc<T>::frag (&a)[KF], const T *Hs, int ldh, int row0,
                                                  const float *b2s)
{
    typedef typename Mc<T>::frag frag;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    const T *hrow = Hs + (row0 + lr) * ldh + 8 * lh;
    mc_floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    frag b[3];
    b[0] = *reinterpret_cast<const frag *>(hrow);
    if (KF > 1) b[1] = *reinterpret_cast<const frag *>(hrow + 16);
#pragma unroll
    for (int kf = 0; kf < KF; ++kf) {
        if (kf + 2 < KF) b[(kf + 2) % 3] = *reinterpret_cast<const frag *>(hrow + (kf + 2) * 16);
        __builtin_amdgcn_sched_barrier(0);
        acc = Mc<T>::mma(a[kf], b[kf % 3], acc);
        __builtin_amdgcn_sched_barrier(0);
    }
    // D[i][j]: i = output (row of W2), j = staged row; lane = j + 32*((i/4)%2), register = i%4 + 4*(i/8)
    const float4 *bv = reinterpret_cast<const float4 *>(b2s + wave * 32 + 4 * lh);   // outputs 8q + 4 lh + 0..3
    float abs_sum = 0.0f, prod = 1.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) eloc_logcosh4(acc, q, bv[2 * q], abs_sum, prod);
    // 16 factors in (1, 2]: the product stays below 2^16
    float s = abs_sum + __logf(prod) - 16.0f * kLn2f;
    s += __shfl_xor(s, 32, 64);
    return s;
}

// ---------------------------------------------------------------------------
// Sampler
// ---------------------------------------------------------------------------
template <typename T>
struct RegSampleLds {
    static __host__ __device__ size_t bytes(int N, int KE, int m2p)
    {
        const size_t K = 16 * (size_t)KE, ldh = K + hs_pad<T>();
        const int NW = (N + 31) / 32;
        size_t b = 0;
        b += sizeof(T) * (size_t)N * K;                       // W1 columns
        b += sizeof(T) * (size_t)(kRegRows + 1) * ldh;        // h1 rows (+1: where ineffective proposals go)
        b += sizeof(float) * m2p;                             // b2
        b += sizeof(float) * K;                               // b1 minus the W1 row sums
        b += sizeof(float) * kRegWaves * kRegRows;            // partial sums
        b += sizeof(uint32_t) * (size_t)kRegRows * NW;        // spin words
        b += sizeof(int) * 4 + 16;                            // slot counters
        return b;
    }
};

// a.lo * b.lo + a.hi * b.hi + c for two 16-bit values packed in a 32-bit word, on the 16-bit dot instruction;
// pair(x, y) packs two values that the format holds exactly (0 and 1 here)
template <typename T>
struct Dot2;
template <>
struct Dot2<__bf16> {
    typedef __bf16 v2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ uint32_t pair(float lo, float hi)
    {
        return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xFFFF0000u);
    }
    static __device__ __forceinline__ float dot(uint32_t a, uint32_t b, float c)
    {
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2, a), __builtin_bit_cast(v2, b), c, false);
    }
};
template <>
struct Dot2<_Float16> {
    typedef _Float16 v2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ uint32_t pair(float lo, float hi)
    {
        return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)lo) |
               ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)hi) << 16);
    }
    static __device__ __forceinline__ float dot(uint32_t a, uint32_t b, float c)
    {
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(v2, a), __builtin_bit_cast(v2, b), c, false);
    }
};

// Each wave owns 8 chains: it draws their proposals (lanes 0..7), stages the
// effective ones at slots taken from a shared counter, and after the matrix
// product decides them and updates their state.  Two barriers per step: after
// the staging (h1 rows complete) and after the product (partial sums complete).
template <typename T, int KE, bool TRACE, bool PERCHAIN>
__global__ void __launch_bounds__(kRegThreads) ffnn_sample_reg_kernel(FfnnSampleArgs A)
{
    typedef typename Mc<T>::frag frag;
    constexpr int K = 16 * KE;                      // hidden units multiplied (KE = ceil(m1 / 16) fragments)
    constexpr int NCH = K / 8;                      // 8-unit chunks: lane c owns units 8c .. 8c + 7
    constexpr int RPW = kRegRows / kRegWaves;       // chains per wave (8)
    extern __shared__ __align__(16) unsigned char smem[];
    const FfnnDev &net = A.net;
    const int N = net.widths[0], m1p = net.m1p, m2p = net.m2p, m2 = net.widths[2];
    const int NW = (N + 31) >> 5;
    const int ldh = K + hs_pad<T>();
    const int nwt = (m2 + 31) >> 5;                 // waves that own real outputs
    T *W1l = reinterpret_cast<T *>(smem);           // [N][K]
    T *Hs = W1l + (size_t)N * K;                    // [kRegRows + 1][ldh]
    float *b2s = reinterpret_cast<float *>(Hs + (size_t)(kRegRows + 1) * ldh);
    float *b1c = b2s + m2p;                         // [K] b1 - sum_i W1[:, i]
    float *part = b1c + K;
    uint32_t *words = reinterpret_cast<uint32_t *>(part + kRegWaves * kRegRows);
    int *cnt = reinterpret_cast<int *>(words + kRegRows * NW);   // [4] rows and live chains of this / the next round

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kRegRows;
    const int nvalid = (int)min<int64_t>(kRegRows, A.n_chains - c0);
    const int myrow = wave * RPW + (lane & (RPW - 1));           // the chain of proposal lanes 0..7
    const bool plane = lane < RPW && myrow < nvalid;
    const int c8 = 8 * (lane < NCH ? lane : NCH - 1);   // this lane's units (lanes past the last chunk repeat it)
    const bool live = __builtin_amdgcn_readfirstlane(wave) * 32 < m2;   // this wave owns real outputs

    frag a[KE];
    reg_load_w2<T, KE>(reinterpret_cast<const T *>(A.W2), m1p, m2p, a);
    {
        const T *src = reinterpret_cast<const T *>(A.W1t);
        for (int k = tid; k < N * NCH; k += kRegThreads) {
            const int i = k / NCH, c = k % NCH;
            *reinterpret_cast<frag *>(W1l + i * K + 8 * c) = *reinterpret_cast<const frag *>(src + (size_t)i * m1p + 8 * c);
        }
        for (int k = tid; k < (kRegRows + 1) * ldh; k += kRegThreads) Hs[k] = Mc<T>::from_f32(0.0f);
        for (int k = tid; k < m2p; k += kRegThreads) b2s[k] = net.b2p[k];
        for (int k = tid; k < kRegRows * NW; k += kRegThreads) {
            const int r = k / NW, w = k % NW;
            uint32_t bits = 0;
            if (r < nvalid) {
                const int8_t *s = A.chain_state + (c0 + r) * N + 32 * w;
                const int nb = min(32, N - 32 * w);
                for (int b = 0; b < nb; ++b) bits |= (s[b] > 0 ? 1u : 0u) << b;
            }
            words[k] = bits;
        }
        if (tid < 4) cnt[tid] = 0;
    }
    __syncthreads();
    for (int u = tid; u < K; u += kRegThreads) {
        float sum = 0.0f;
        for (int i = 0; i < N; ++i) sum += Mc<T>::to_f32(W1l[i * K + u]);
        b1c[u] = net.b1p[u] - sum;
    }
    __syncthreads();

    float z1[RPW][8];
    // z1 = W1 s + b1 of the wave's chains r in `mask` (bit r; wave-uniform), as (b1 - sum_i W1[:, i]) plus twice
    // the sum of W1[:, i] over the chain's up spins: half the columns of a sum over all sites.  The up spins are
    // taken in site order, four W1 columns read ahead of their use (a missing one weighted by 0), and two
    // columns at a time added on the 16-bit dot instruction (each unit's pair of weights by the pair of weights
    // 0 or 1, in FP32).
    auto refresh_rows = [&](unsigned mask) {
        const float4 cb0 = *reinterpret_cast<const float4 *>(b1c + c8);
        const float4 cb1 = *reinterpret_cast<const float4 *>(b1c + c8 + 4);
        const float cb[8] = {cb0.x, cb0.y, cb0.z, cb0.w, cb1.x, cb1.y, cb1.z, cb1.w};
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            if (!((mask >> r) & 1u)) continue;
            float up[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            for (int wi = 0; wi < NW; ++wi) {
                uint32_t bits = __builtin_amdgcn_readfirstlane(words[(wave * RPW + r) * NW + wi]);
                while (bits) {
                    int idx[4];
                    float m[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        m[u] = bits ? 1.0f : 0.0f;
                        idx[u] = bits ? 32 * wi + __builtin_ctz(bits) : 0;
                        bits &= bits - 1u;
                    }
                    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
                    u32x4_t w[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) w[u] = *reinterpret_cast<const u32x4_t *>(W1l + idx[u] * K + c8);
#pragma unroll
                    for (int u = 0; u < 4; u += 2) {
                        const uint32_t mp = Dot2<T>::pair(m[u], m[u + 1]);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            // (unit 2k of columns u, u + 1), (unit 2k + 1 of columns u, u + 1)
                            up[2 * k] = Dot2<T>::dot(__builtin_amdgcn_perm(w[u + 1][k], w[u][k], 0x05040100u), mp, up[2 * k]);
                            up[2 * k + 1] =
                                Dot2<T>::dot(__builtin_amdgcn_perm(w[u + 1][k], w[u][k], 0x07060302u), mp, up[2 * k + 1]);
                        }
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) z1[r][e] = fmaf(2.0f, up[e], cb[e]);
        }
    };
    constexpr unsigned kAllRows = (1u << RPW) - 1u;
    // layer-1 change of flipping i (and j >= 0) where site i holds spin si (no branch: W1[:, max(j, 0)] is read
    // and weighted by 0 for a flip, which leaves W1[:, i] exact)
    auto delta_z1 = [&](int i, int j, float si, float (&dz)[8]) {
        const float g = -2.0f * si, jm = j >= 0 ? 1.0f : 0.0f;
        const frag wi = *reinterpret_cast<const frag *>(W1l + i * K + c8);
        const frag wj = *reinterpret_cast<const frag *>(W1l + (j >= 0 ? j : 0) * K + c8);
#pragma unroll
        for (int e = 0; e < 8; ++e) dz[e] = g * fmaf(-jm, Mc<T>::to_f32(wj[e]), Mc<T>::to_f32(wi[e]));
    };
    // h1 = ReLU(z + dz) of one row, this lane's 8 units
    auto store_row = [&](int row, const float (&z)[8], const float (&dz)[8]) {
        frag h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = Mc<T>::from_f32(fmaxf(z[e] + dz[e], 0.0f));
        *reinterpret_cast<frag *>(Hs + row * ldh + c8) = h;
    };
    // log|psi| of this wave's chains from the current z1 (lanes 0..7 return their chain's value)
    auto full_eval = [&]() -> float {
        const float zero[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < RPW; ++r) store_row(wave * RPW + r, z1[r], zero);
        __syncthreads();
        if (live)
            for (int t = 0; t < kRegRows / 32; ++t) {
                const float s = reg_tile_logcosh<T, KE>(a, Hs, ldh, 32 * t, b2s);
                if (lane < 32) part[wave * kRegRows + 32 * t + lane] = s;
            }
        __syncthreads();
        float f = 0.0f;
        for (int w = 0; w < nwt; ++w) f += part[w * kRegRows + myrow];
        return f;
    };

    refresh_rows(kAllRows);
    float fcur = full_eval();   // meaningful on proposal lanes

    unsigned long long acc = 0;   // accepted proposals of this lane's chain
    if constexpr (PERCHAIN) {
        // Each chain advances through its own steps.  Per round (two barriers) a chain draws proposals until one
        // changes its state: the others (an exchange of equal spins) are accepted without an evaluation, so
        // they are decided on the spot.  It stops early at the end of a sweep, where its sample is written out;
        // at the ends of sweeps that refresh z1 it recomputes z1 and evaluates its current state in the next
        // tile instead of a proposal, before that sample is written.  The rows of a round are those proposals
        // and refreshes (compacted), so the tiles are full however many proposals were ineffective; every
        // decision, value and output equals that of all chains stepping together.
        const int sw = A.sweep_size;
        const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * sw;
        const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
        int64_t kc = 0;              // the chain's next step (proposal lanes)
        int in_sweep = 0, sweep = 0; // steps done in the current sweep; sweeps completed
        bool need_refresh = false;   // z1 and f are recomputed before the pending sample is written
        int emit_q = -1;             // sweep whose sample is still to be written
        int par = 0;
        int64_t rounds = 0;
        // the decision of an ineffective proposal (its log-ratio is 0)
        auto trace = [&](int64_t k, int pi_, int pj_, uint32_t ub_, float d2, bool accept) {
            if constexpr (TRACE) {
                const int64_t c = c0 + myrow;
                if (c < A.n_traced) {
                    const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                    A.tr_site[idx] = pi_ | ((pj_ < 0 ? 0xFFFF : pj_) << 16);
                    A.tr_ubits[idx] = ub_;
                    A.tr_delta[idx] = d2 * kLn2f;
                    A.tr_acc[idx] = accept ? 1 : 0;
                }
            }
        };
        // a step has been decided: at the end of a sweep its sample is due, after a refresh when one is due
        auto end_of_step = [&]() {
            if (++in_sweep == sw) {
                in_sweep = 0;
                emit_q = sweep++;
                need_refresh = sweep % A.refresh_sweeps == 0;
            }
        };
        while (true) {
            // proposals of this wave's chains: mode 1 an effective proposal, 2 a refresh row.  The next 8 steps of
            // chain r are drawn at once by lanes 8r .. 8r + 7 (lane 8r + d: step kc + d, up to the end of the sweep
            // and of the call); the steps before the first effective one are ineffective and decided on the spot.
            const int gr = lane >> 3, gd = lane & 7;                    // chain and look-ahead of this lane
            const int64_t kc_g = ((int64_t)__shfl(int(kc >> 32), gr, 64) << 32) | (uint32_t)__shfl(int(kc), gr, 64);
            const int in_g = __shfl(in_sweep, gr, 64);
            const bool search = plane && !need_refresh && emit_q < 0 && kc < total;
            const bool search_g = __shfl(search ? 1 : 0, gr, 64) != 0;
            const int64_t left_g = total - kc_g;
            const int lim_g = (int)min<int64_t>(min<int64_t>(8, left_g), (int64_t)(sw - in_g));   // steps of the window
            const bool inwin = search_g && gd < lim_g;
            int wpi = 0, wpj = -1;
            uint32_t wub = 0;
            bool wup = false, weff = false;
            if (inwin) {
                const uint64_t step = A.step_offset + (uint64_t)(kc_g + gd);
                const uint32_t gidg = A.chain_id_offset + (uint32_t)(c0 + wave * RPW + gr);
                const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gidg, A.inst << 8, key0, key1);
                wpi = index_from_word(rb.r0, N);
                if (A.move == 1) {
                    wpj = index_from_word(rb.r1, N - 1);
                    wpj += (wpj >= wpi) ? 1 : 0;
                }
                const uint32_t *w = words + (wave * RPW + gr) * NW;
                wup = (w[wpi >> 5] >> (wpi & 31)) & 1u;
                weff = wpj < 0 || wup != (bool)((w[wpj >> 5] >> (wpj & 31)) & 1u);
                wub = rb.r2 >> 8;
            }
            const unsigned long long effb = __ballot(weff);
            const unsigned gbits = (unsigned)(effb >> (8 * gr)) & 0xFFu;
            const int first_g = gbits ? __builtin_ctz(gbits) : 8;        // look-ahead of the first effective step
            // ineffective steps before it: log-ratio 0, accepted when log2 u < 0
            const bool skip = inwin && gd < first_g;
            bool skip_acc = false;
            if (skip) {
                const float l2u = __builtin_amdgcn_logf((float)wub * 5.9604644775390625e-8f);
                skip_acc = l2u < 0.0f;
                if constexpr (TRACE) {
                    const int64_t c = c0 + wave * RPW + gr;
                    if (c < A.n_traced) {
                        const size_t idx = (size_t)c * (size_t)total + (size_t)(kc_g + gd);
                        A.tr_site[idx] = wpi | ((wpj < 0 ? 0xFFFF : wpj) << 16);
                        A.tr_ubits[idx] = wub;
                        A.tr_delta[idx] = 0.0f;
                        A.tr_acc[idx] = skip_acc ? 1 : 0;
                    }
                }
            }
            const unsigned long long accb = __ballot(skip_acc);
            // the window's outcome for chain r = lane (lanes 0..7): the look-ahead of its first effective step
            // (from the ballot) and the window's length (from the chain's own counters), then the effective
            // proposal from lane 8r + first, shuffled with every lane active (a shuffle from an inactive lane
            // returns 0)
            const unsigned cbits = (unsigned)(effb >> (8 * (lane & 7))) & 0xFFu;
            const int first_c = cbits ? __builtin_ctz(cbits) : 8;
            const int lim_c = (int)min<int64_t>(min<int64_t>(8, total - kc), (int64_t)(sw - in_sweep));
            const int src = 8 * (lane & 7) + min(first_c, 7);
            const int e_pi = __shfl(wpi, src, 64), e_pj = __shfl(wpj, src, 64);
            const uint32_t e_ub = (uint32_t)__shfl((int)wub, src, 64);
            const bool e_up = __shfl(wup ? 1 : 0, src, 64) != 0;
            int pi = 0, pj = -1, slot = -1, mode = 0;
            float si = 0.0f;   // 0 leaves a refresh row (or no row) without a layer-1 change
            uint32_t ub = 0;
            if (plane) {
                if (need_refresh) {
                    mode = 2;
                } else if (search) {
                    const int first = first_c, lim = lim_c;
                    const int nskip = min(first, lim);
                    acc += (unsigned long long)__popc((unsigned)(accb >> (8 * lane)) & 0xFFu);
                    kc += nskip;
                    in_sweep += nskip;
                    if (in_sweep == sw) {   // the sweep ended on ineffective steps
                        in_sweep = 0;
                        emit_q = sweep++;
                        need_refresh = sweep % A.refresh_sweeps == 0;
                        if (need_refresh) mode = 2;   // the refresh row goes in this round
                    } else if (first < lim) {
                        pi = e_pi;
                        pj = e_pj;
                        ub = e_ub;
                        si = e_up ? 1.0f : -1.0f;
                        mode = 1;
                    }
                }
                if (mode != 0) slot = atomicAdd(&cnt[par], 1);
            }
            // chains that refresh: z1 recomputed from their spins
            const unsigned rm = (unsigned)__ballot(mode == 2) & kAllRows;
            if (rm) refresh_rows(rm);
            // stage the rows (wave-uniform per chain): every chain's row is formed, one without a row goes to the
            // spare row kRegRows, so that the code has no branch and later reads overlap earlier stores
    #pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int sl = __builtin_amdgcn_readlane(slot, r);
                const int i = __builtin_amdgcn_readlane(pi, r), j = __builtin_amdgcn_readlane(pj, r);
                const float s_i = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(si), r));
                float dz[8];
                delta_z1(i, j, s_i, dz);
                store_row(sl >= 0 ? sl : kRegRows, z1[r], dz);
            }
            // chains with work left are counted with the rows: none left ends the call for the whole block
            if (plane && (kc < total || need_refresh || emit_q >= 0)) atomicAdd(&cnt[2 + par], 1);
            __syncthreads();
            // every live chain advances each round (a step, a refresh or a sample written), so this count reaches
            // zero within 3 total + 2 rounds; the bound only makes that explicit
            if (cnt[2 + par] == 0 || ++rounds > 3 * total + 2) break;
            const int neff = cnt[par];
            for (int t = 0; live && 32 * t < neff; ++t) {
                const float s = reg_tile_logcosh<T, KE>(a, Hs, ldh, 32 * t, b2s);
                if (lane < 32) part[wave * kRegRows + 32 * t + lane] = s;
            }
            if (tid == 0) {   // read next in the following round, after the barrier below
                cnt[par ^ 1] = 0;
                cnt[2 + (par ^ 1)] = 0;
            }
            __syncthreads();
            // decisions and refreshed values of this wave's chains
            bool upd = false;
            if (plane && mode != 0) {
                float fnew = 0.0f;
                for (int w = 0; w < nwt; ++w) fnew += part[w * kRegRows + slot];
                if (mode == 2) {
                    fcur = fnew;
                    need_refresh = false;
                } else {
                    const float d2 = 2.0f * (fnew - fcur) / kLn2f;
                    const float l2u = __builtin_amdgcn_logf((float)ub * 5.9604644775390625e-8f);
                    const bool accept = l2u < d2;   // NaN rejects
                    if (accept) ++acc;
                    upd = accept;
                    if (upd) {
                        uint32_t *w = words + myrow * NW;
                        w[pi >> 5] ^= 1u << (pi & 31);
                        if (pj >= 0) w[pj >> 5] ^= 1u << (pj & 31);
                        fcur = fnew;
                    }
                    trace((int64_t)kc, pi, pj, ub, d2, accept);
                    ++kc;
                    end_of_step();
                }
            }
            // apply the accepted moves to z1
            const unsigned long long um = __ballot(upd);
    #pragma unroll
            for (int r = 0; r < RPW; ++r) {
                if ((um >> r) & 1ull) {
                    const int i = __builtin_amdgcn_readlane(pi, r), j = __builtin_amdgcn_readlane(pj, r);
                    const float s_i = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(si), r));
                    float dz[8];
                    delta_z1(i, j, s_i, dz);
    #pragma unroll
                    for (int e = 0; e < 8; ++e) z1[r][e] += dz[e];
                }
            }
            // samples due (no refresh pending): the chain's spins and log|psi|
            const bool emit = plane && emit_q >= 0 && !need_refresh;
            const unsigned long long em = __ballot(emit);
            const int out_lane = emit_q - A.n_burnin;
    #pragma unroll
            for (int r = 0; r < RPW; ++r) {
                if ((em >> r) & 1ull) {
                    const int out = __builtin_amdgcn_readlane(out_lane, r);
                    const int row = wave * RPW + r;
                    if (out >= 0 && A.samples)
                        for (int i = lane; i < N; i += 64)
                            A.samples[((size_t)out * A.n_chains + c0 + row) * N + i] =
                                ((words[row * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1 : -1;
                }
            }
            if (emit) {
                if (out_lane >= 0 && A.logpsi) A.logpsi[(size_t)out_lane * A.n_chains + c0 + myrow] = fcur;
                emit_q = -1;
            }
            par ^= 1;
        }
    } else {
        // All chains step together: one proposal per chain per step, the effective ones evaluated.
        const int sw = A.sweep_size;
        const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * sw;
        const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
        int in_sweep = 0, since_refresh = 0;
        int64_t sweep = 0;
        for (int64_t k = 0; k < total; ++k) {
            // proposals of this wave's chains (lanes 0..7); effective ones take a slot
            int pi = 0, pj = -1, slot = -1;
            float si = 1.0f;
            uint32_t ub = 0;
            if (plane) {
                const uint64_t step = A.step_offset + (uint64_t)k;
                const uint32_t gid = A.chain_id_offset + (uint32_t)(c0 + myrow);
                const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, A.inst << 8, key0, key1);
                pi = index_from_word(rb.r0, N);
                if (A.move == 1) {
                    pj = index_from_word(rb.r1, N - 1);
                    pj += (pj >= pi) ? 1 : 0;
                }
                const uint32_t *w = words + myrow * NW;
                const bool up = (w[pi >> 5] >> (pi & 31)) & 1u;
                si = up ? 1.0f : -1.0f;
                const bool eff = pj < 0 || up != (bool)((w[pj >> 5] >> (pj & 31)) & 1u);
                if (eff) slot = atomicAdd(&cnt[k & 1], 1);
                ub = rb.r2 >> 8;
            }
            // stage h1 of the effective proposals (rows are wave-uniform); every chain's row is formed and an
            // ineffective one goes to the spare row kRegRows, so that the code has no branch and the reads of later
            // chains can be issued before earlier rows are stored
    #pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int sl = __builtin_amdgcn_readlane(slot, r);
                const int i = __builtin_amdgcn_readlane(pi, r), j = __builtin_amdgcn_readlane(pj, r);
                const float s_i = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(si), r));
                float dz[8];
                delta_z1(i, j, s_i, dz);
                store_row(sl >= 0 ? sl : kRegRows, z1[r], dz);
            }
            __syncthreads();
            const int neff = cnt[k & 1];
            for (int t = 0; live && 32 * t < neff; ++t) {
                const float s = reg_tile_logcosh<T, KE>(a, Hs, ldh, 32 * t, b2s);
                if (lane < 32) part[wave * kRegRows + 32 * t + lane] = s;
            }
            if (tid == 0) cnt[(k + 1) & 1] = 0;   // read next in step k + 1, after the barrier below
            __syncthreads();
            // decisions of this wave's chains
            bool upd = false;
            if (plane) {
                float fnew = 0.0f;
                if (slot >= 0)
                    for (int w = 0; w < nwt; ++w) fnew += part[w * kRegRows + slot];
                const float d2 = slot >= 0 ? 2.0f * (fnew - fcur) / kLn2f : 0.0f;
                const float l2u = __builtin_amdgcn_logf((float)ub * 5.9604644775390625e-8f);
                const bool accept = l2u < d2;   // NaN rejects
                if (accept) ++acc;
                upd = accept && slot >= 0;
                if (upd) {
                    uint32_t *w = words + myrow * NW;
                    w[pi >> 5] ^= 1u << (pi & 31);
                    if (pj >= 0) w[pj >> 5] ^= 1u << (pj & 31);
                    fcur = fnew;
                }
                if constexpr (TRACE) {
                    const int64_t c = c0 + myrow;
                    if (c < A.n_traced) {
                        const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                        A.tr_site[idx] = pi | ((pj < 0 ? 0xFFFF : pj) << 16);
                        A.tr_ubits[idx] = ub;
                        A.tr_delta[idx] = d2 * kLn2f;
                        A.tr_acc[idx] = accept ? 1 : 0;
                    }
                }
            }
            // apply the accepted moves to z1
            const unsigned long long um = __ballot(upd);
    #pragma unroll
            for (int r = 0; r < RPW; ++r) {
                if ((um >> r) & 1ull) {
                    const int i = __builtin_amdgcn_readlane(pi, r), j = __builtin_amdgcn_readlane(pj, r);
                    const float s_i = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(si), r));
                    float dz[8];
                    delta_z1(i, j, s_i, dz);
    #pragma unroll
                    for (int e = 0; e < 8; ++e) z1[r][e] += dz[e];
                }
            }
            if (++in_sweep == sw) {
                in_sweep = 0;
                const int64_t out = sweep - A.n_burnin;
                if (++since_refresh == A.refresh_sweeps) {
                    refresh_rows(kAllRows);
                    const float f = full_eval();
                    if (plane) fcur = f;
                    since_refresh = 0;
                }
                if (out >= 0) {
                    if (A.samples) {
                        // this wave's chains: lane = site within a word row
                        for (int idx = lane; idx < RPW * N; idx += 64) {
                            const int r = idx / N, i = idx % N, row = wave * RPW + r;
                            if (row < nvalid)
                                A.samples[((size_t)out * A.n_chains + c0 + row) * N + i] =
                                    ((words[row * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1 : -1;
                        }
                    }
                    if (A.logpsi && plane) A.logpsi[(size_t)out * A.n_chains + c0 + myrow] = fcur;
                }
                ++sweep;
            }
        }
    }
    for (int idx = lane; idx < RPW * N; idx += 64) {
        const int r = idx / N, i = idx % N, row = wave * RPW + r;
        if (row < nvalid)
            A.chain_state[(c0 + row) * N + i] = ((words[row * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1 : -1;
    }
    if (A.n_acc && plane) A.n_acc[c0 + myrow] = acc;
}

// ---------------------------------------------------------------------------
// Local energies
//
// The W1 columns the network uses (16 KE hidden units, KE = ceil(m1 / 16)) are
// copied to LDS once per block.  A group of G samples (G <= 8, as many as the
// LDS holds): the block forms z1 = W1 s + b1 of each sample (lane pairs split
// the sites), lists each sample's rows (the sample itself, then its connected
// configurations) and evaluates the rows of the whole group end to end,
// kElocRows = 32 at a time.  Passes are software-pipelined over two LDS
// buffers of h1 rows: while wave w multiplies its 32 rows of W2 (registers, KE
// fragments of 16) by the current buffer, it stages 4 rows of the next pass
// into the other buffer (lane c: hidden units 8c .. 8c + 7, W1 and z1 read from
// LDS) and, for KE <= 25, turns the previous pass's products into log-cosh
// partials, both written in between the matrix instructions so that they
// overlap them.  One barrier per pass; a pass's row sums over the waves are
// taken one or two passes later.  Waves whose 32 outputs are all padding only
// stage rows.
// ---------------------------------------------------------------------------
constexpr int kElocRows = 32;                        // rows per pass: one 32 x 32 tile per wave
constexpr int kElocStage = kElocRows / kRegWaves;    // rows each wave stages per pass
constexpr int kElocPre = 1;                          // spins of the next group each thread prefetches

template <typename T>
__host__ __device__ inline size_t reg_eloc_lds_bytes(int N, int KE, int m2p, int G)
{
    const size_t K = 16 * (size_t)KE, ldh = K + hs_pad<T>();
    const size_t maxrows = (size_t)G * (2 * N + 1);
    size_t b = 0;
    b += sizeof(T) * (size_t)N * K;                     // W1 columns
    b += sizeof(T) * 2 * (size_t)kElocRows * ldh;       // h1 rows of two passes
    b += sizeof(float) * (size_t)G * K;                 // z1 of the group's samples
    b += sizeof(float) * K;                             // b1
    b += sizeof(float) * m2p;                           // b2
    b += sizeof(float) * 2 * kRegWaves * kElocRows;     // partial sums of two passes
    b += sizeof(float) * (size_t)G * N;                 // spins
    b += sizeof(int) * 2 * (size_t)N;                   // candidate table (flips and bonds)
    b += (sizeof(int) + 3 * sizeof(float)) * maxrows;   // rows: packed (i, j, sample), coefficient, g, f
    b += sizeof(double) * G + sizeof(int) * G + 32;
    return b;
}

// row code: (i + 1) | (j + 1) << 13 | s << 26, i = j = -1 for the sample itself
__device__ __forceinline__ int eloc_row_code(int i, int j, int s) { return (i + 1) | ((j + 1) << 13) | (s << 26); }

// h1 = ReLU(z1 + g (W1[:, i] - W1[:, j])) of row `row` (g = -2 s_i, 0 for the sample's own row; the W1[:, j]
// term only for an exchange), hidden units 8c .. 8c + 7, c = min(lane, nch - 1) (lanes past the row's chunks
// repeat the last one), into Hs row lr.  W1l: [N][K] in LDS; zs: [G][2][K / 8][4] (units 8c .. 8c + 3 of
// every chunk, then units 8c + 4 .. 8c + 7, so that the 16-byte reads of consecutive lanes are consecutive).
// `code` is the row's code, uniform over the wave (read ahead by the caller or from rcode).
template <typename T>
__device__ __forceinline__ void eloc_stage_row_code(const T *W1l, int code, const float *rg, const float *zs,
                                                    T *Hs, int ldh, int K, int nch, int row, int lr, int lane)
{
    typedef typename Mc<T>::frag frag;
    const float g = rg[row];
    const int i = (code & 0x1FFF) - 1, j = ((code >> 13) & 0x1FFF) - 1, s = code >> 26;
    const int ic = i >= 0 ? i : 0, jc = j >= 0 ? j : 0;
    const float jm = j >= 0 ? 1.0f : 0.0f;
    const int c = lane < nch ? lane : nch - 1;
    const frag wi = *reinterpret_cast<const frag *>(W1l + ic * K + 8 * c);
    const frag wj = *reinterpret_cast<const frag *>(W1l + jc * K + 8 * c);
    const float4 z0 = *reinterpret_cast<const float4 *>(zs + s * K + 4 * c);
    const float4 z1 = *reinterpret_cast<const float4 *>(zs + s * K + K / 2 + 4 * c);
    const float zz[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
    frag h;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float d = fmaf(-jm, Mc<T>::to_f32(wj[e]), Mc<T>::to_f32(wi[e]));
        h[e] = Mc<T>::from_f32(fmaxf(fmaf(g, d, zz[e]), 0.0f));
    }
    *reinterpret_cast<frag *>(Hs + lr * ldh + 8 * c) = h;
}

template <typename T>
__device__ __forceinline__ void eloc_stage_row(const T *W1l, const int *rcode, const float *rg, const float *zs,
                                               T *Hs, int ldh, int K, int nch, int row, int lr, int lane)
{
    eloc_stage_row_code<T>(W1l, __builtin_amdgcn_readfirstlane(rcode[row]), rg, zs, Hs, ldh, K, nch, row, lr, lane);
}

template <typename T, int KE>
__global__ void __launch_bounds__(kRegThreads) ffnn_eloc_reg_kernel(FfnnElocArgs A, int G)
{
    typedef typename Mc<T>::frag frag;
    static_assert(KE >= kElocStage, "one staged row every KE / kElocStage fragments");
    constexpr int K = 16 * KE;
    constexpr int NT = kRegThreads, NWV = kRegWaves;
    extern __shared__ __align__(16) unsigned char smem[];
    const FfnnDev &net = A.net;
    const int N = net.widths[0], m1p = net.m1p, m2p = net.m2p, m2 = net.widths[2];
    const int ldh = K + hs_pad<T>();
    const int nwt = (m2 + 31) >> 5;                    // waves with at least one real output
    const int maxrows = G * (2 * N + 1);
    const int nch = K >> 3;                            // 8-unit chunks of a row
    T *W1l = reinterpret_cast<T *>(smem);              // [N][K]
    T *Hs = W1l + (size_t)N * K;                       // [2][kElocRows][ldh]
    float *zs = reinterpret_cast<float *>(Hs + 2 * (size_t)kElocRows * ldh);   // [G][2][K / 8][4]
    float *b1s = zs + (size_t)G * K;                   // [K]
    float *b2s = b1s + K;                              // [m2p]
    float *part = b2s + m2p;                           // [2][kRegWaves][kElocRows]
    float *sp = part + 2 * kRegWaves * kElocRows;      // [G][N]
    int *ctab = reinterpret_cast<int *>(sp + (size_t)G * N);   // [2N]
    int *rcode = ctab + 2 * N;                         // [maxrows]
    float *rc = reinterpret_cast<float *>(rcode + maxrows);
    float *rg = rc + maxrows;
    float *fr = rg + maxrows;
    // (an offset from smem, not an integer cast of the pointer, so that the compiler keeps the LDS address space)
    const size_t diag_off = ((size_t)(reinterpret_cast<unsigned char *>(fr + maxrows) - smem) + 7) & ~(size_t)7;
    double *diag = reinterpret_cast<double *>(smem + diag_off);
    int *rcnt = reinterpret_cast<int *>(diag + G);     // [G]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const int lr = lane & 31, lh = lane >> 5;
    const bool live = wave_u * 32 < m2;                // this wave owns real outputs
    const bool late_phase = (wave_u >> 2) & 1;         // the second wave on a SIMD runs its pass shifted
    frag a[KE];
    reg_load_w2<T, KE>(reinterpret_cast<const T *>(A.W2), m1p, m2p, a);
    {
        const T *src = reinterpret_cast<const T *>(A.W1t);
        for (int k = tid; k < N * nch; k += NT) {
            const int i = k / nch, c = k % nch;
            *reinterpret_cast<frag *>(W1l + i * K + 8 * c) = *reinterpret_cast<const frag *>(src + (size_t)i * m1p + 8 * c);
        }
    }
    for (int k = tid; k < K; k += NT) b1s[k] = net.b1p[k];
    for (int k = tid; k < m2p; k += NT) b2s[k] = net.b2p[k];
    const int nb = A.dim == 1 ? (A.pbc ? A.L : A.L - 1) : 2 * A.L * A.L;   // candidate bonds (2D: 2 per site)
    const int ncand = A.kind == NQS_TFIM ? N : 0;
    const int nloop = ncand > nb ? ncand : nb;
    // candidate table: bond c as (bi + 1) | (bj + 1) << 13 | sign flip of the Marshall rule << 26 (0: no bond),
    // and the Marshall sign of flipping site c << 27
    for (int c = tid; c < nloop; c += NT) {
        int t = 0;
        if (c < nb) {
            int bi, bj;
            bool valid = true;
            if (A.dim == 1) {
                bi = c;
                bj = c + 1 < A.L ? c + 1 : 0;
            } else {
                const int site = c >> 1, x = site / A.L, y = site % A.L;
                bi = site;
                if ((c & 1) == 0) {
                    valid = A.pbc || x + 1 < A.L;
                    bj = ((x + 1) % A.L) * A.L + y;
                } else {
                    valid = A.pbc || y + 1 < A.L;
                    bj = x * A.L + (y + 1) % A.L;
                }
            }
            const bool flip = A.marshall && (on_sub_a(A.dim, A.L, bi) != on_sub_a(A.dim, A.L, bj));
            if (valid) t = (bi + 1) | ((bj + 1) << 13) | ((flip ? 1 : 0) << 26);
        }
        if (c < ncand && A.marshall && on_sub_a(A.dim, A.L, c)) t |= 1 << 27;
        ctab[c] = t;
    }

    // candidate c of a sample: a flip (TFIM) and / or a bond; returns whether it gives a row
    auto candidate = [&](const float *ss, int c, int &i, int &j, float &coef, double &dg) {
        const int t = ctab[c];
        bool take = false;
        i = -1;
        j = -1;
        coef = 0.0f;
        if (c < ncand) {
            i = c;
            take = true;
            coef = (float)A.h * (((t >> 27) & 1) ? -1.0f : 1.0f);
        }
        const int bi = (t & 0x1FFF) - 1;
        if (bi >= 0) {
            const int bj = ((t >> 13) & 0x1FFF) - 1;
            dg += A.J * (double)(ss[bi] * ss[bj]);
            if (A.kind == NQS_HEISENBERG && ss[bi] != ss[bj]) {
                i = bi;
                j = bj;
                take = true;
                coef = 2.0f * (float)A.J * (((t >> 26) & 1) ? -1.0f : 1.0f);
            }
        }
        return take;
    };
    // f of the rows of pass q: the sum of the waves' partials (in wave order)
    auto row_sums = [&](int q, int nrows) {
        if (tid < kElocRows && q * kElocRows + tid < nrows) {
            const float *pp = part + (size_t)(q & 1) * kRegWaves * kElocRows;
            float f = 0.0f;
            for (int w = 0; w < nwt; ++w) f += pp[w * kElocRows + tid];
            fr[q * kElocRows + tid] = f;
        }
    };
    // the log-cosh partial of a finished tile: sum_k log cosh z2 = sum |z2| + log prod (1 + e^-2|z2|) - n ln 2
    // (16 factors in (1, 2]: the product stays below 2^16; padded outputs have z2 = 0 exactly and add 0)
    auto finish_tile = [&](float abs_sum, float prod, int q) {
        float sv = abs_sum + __logf(prod) - 16.0f * kLn2f;
        sv += __shfl_xor(sv, 32, 64);
        if (lane < 32) part[(size_t)(q & 1) * kRegWaves * kElocRows + wave * kElocRows + lane] = sv;
    };
    const float4 *b2v = reinterpret_cast<const float4 *>(b2s + wave * 32 + 4 * lh);   // outputs 8q + 4 lh + 0..3

    // spins of a group: the first directly, each later one from the registers loaded during the previous group
    int8_t pre[kElocPre];
    auto prefetch = [&](int64_t gs, int ngs) {
#pragma unroll
        for (int m = 0; m < kElocPre; ++m) {
            const int k = tid + m * NT;
            pre[m] = (k < G * N && k / N < ngs) ? A.samples[(gs + k / N) * N + k % N] : (int8_t)1;
        }
    };
    bool have_pre = false;
    for (int64_t g0 = (int64_t)blockIdx.x * G; g0 < A.n; g0 += (int64_t)gridDim.x * G) {
        const int ns = (int)min<int64_t>(G, A.n - g0);
        __syncthreads();   // the previous group's rows and energies are consumed (and the tables are in place)
        for (int k = tid; k < G * N; k += NT) {
            const int s = k / N, i = k % N, m = k / NT;
            sp[k] = have_pre && m < kElocPre ? (float)pre[m] : (s < ns ? (float)A.samples[(g0 + s) * N + i] : 1.0f);
        }
        __syncthreads();
        {
            const int64_t gn = g0 + (int64_t)gridDim.x * G;
            have_pre = gn < A.n;
            if (have_pre) prefetch(gn, (int)min<int64_t>(G, A.n - gn));
        }
        // z1 = W1 s + b1: task (sample, chunk) per lane pair, lane l + 32 h sums the sites of half h
        for (int q = wave * 32 + lr; q < G * nch; q += NWV * 32) {
            const int s = q / nch, c = q % nch;
            const float *ss = sp + s * N;
            float z[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) z[e] = 0.0f;
            const int i0 = lh ? N / 2 : 0, i1 = lh ? N : N / 2;
#pragma unroll 4
            for (int i = i0; i < i1; ++i) {
                const frag w = *reinterpret_cast<const frag *>(W1l + i * K + 8 * c);
                const float sv = ss[i];
#pragma unroll
                for (int e = 0; e < 8; ++e) z[e] = fmaf(Mc<T>::to_f32(w[e]), sv, z[e]);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) z[e] += __shfl_xor(z[e], 32, 64);
            if (lh == 0) {
                const float4 c0 = *reinterpret_cast<const float4 *>(b1s + 8 * c);
                const float4 c1 = *reinterpret_cast<const float4 *>(b1s + 8 * c + 4);
                *reinterpret_cast<float4 *>(zs + s * K + 4 * c) =
                    make_float4(z[0] + c0.x, z[1] + c0.y, z[2] + c0.z, z[3] + c0.w);
                *reinterpret_cast<float4 *>(zs + s * K + K / 2 + 4 * c) =
                    make_float4(z[4] + c1.x, z[5] + c1.y, z[6] + c1.z, z[7] + c1.w);
            }
        }
        // wave s: its sample's row count and diagonal part
        if (wave < ns) {
            const float *ss = sp + wave * N;
            double dg = 0.0;
            int cnt = 0;
            for (int c0 = 0; c0 < nloop; c0 += 64) {
                int i, j;
                float coef;
                const bool take = c0 + lane < nloop && candidate(ss, c0 + lane, i, j, coef, dg);
                cnt += __popcll(__ballot(take));
            }
            dg = group_sum<64>(dg);
            if (lane == 0) {
                rcnt[wave] = cnt;
                diag[wave] = dg;
            }
        }
        __syncthreads();
        // the group's rows, sample after sample (every thread forms the offsets from the counts)
        int nrows = 0, r0 = 0;
        for (int s = 0; s < ns; ++s) {
            if (s == wave) r0 = nrows;
            nrows += 1 + rcnt[s];
        }
        // wave s: the rows of its sample, in candidate order after the sample's own row
        if (wave < ns) {
            const float *ss = sp + wave * N;
            if (lane == 0) {
                rcode[r0] = eloc_row_code(-1, -1, wave);
                rc[r0] = 0.0f;
                rg[r0] = 0.0f;
            }
            int pos0 = r0 + 1;
            double unused = 0.0;
            for (int c0 = 0; c0 < nloop; c0 += 64) {
                int i, j;
                float coef;
                const bool take = c0 + lane < nloop && candidate(ss, c0 + lane, i, j, coef, unused);
                const unsigned long long bal = __ballot(take);
                if (take) {
                    const int pos = pos0 + __popcll(bal & ((1ull << lane) - 1ull));
                    rcode[pos] = eloc_row_code(i, j, wave);
                    rc[pos] = coef;
                    rg[pos] = -2.0f * ss[i];
                }
                pos0 += __popcll(bal);
            }
        }
        __syncthreads();
        const int npass = (nrows + kElocRows - 1) / kElocRows;
        // wave w stages rows w kElocStage .. w kElocStage + kElocStage - 1 of pass q into buffer q & 1 (rows
        // past the group's end are clamped copies that nothing reads)
        auto stage_pass = [&](int q) {
            T *Hq = Hs + (size_t)(q & 1) * kElocRows * ldh;
#pragma unroll
            for (int rr = 0; rr < kElocStage; ++rr) {
                const int r = wave * kElocStage + rr;
                eloc_stage_row<T>(W1l, rcode, rg, zs, Hq, ldh, K, nch, min(q * kElocRows + r, nrows - 1), r, lane);
            }
        };
        stage_pass(0);
        __syncthreads();
        // one pass of a multiplying wave: its 32 outputs for the 32 rows of pass p, each B fragment read two
        // products ahead of its use (the order pinned against the scheduler), with its kElocStage rows of pass
        // p + 1 staged in between the products, then the tile's log-cosh partial.  The two waves that share a
        // SIMD (w and w + 4) place their staging slots half a period apart (PH), so that one of them issues
        // products while the other stages.
        // the codes of a wave's staging rows are read from LDS one pass ahead (across the barrier) and taken
        // into scalar registers at the start of the pass, so that a staging slot waits for one LDS round trip
        // (its W1 columns, z1 and g), not two
        auto read_codes = [&](int q, int (&cv)[kElocStage]) {
#pragma unroll
            for (int rr = 0; rr < kElocStage; ++rr) cv[rr] = rcode[min(q * kElocRows + wave * kElocStage + rr, nrows - 1)];
        };
        int cv[kElocStage];
        read_codes(1, cv);
        auto pass = [&](int p, auto ph_c) {
            constexpr bool PH = decltype(ph_c)::value;
            int code[kElocStage];
#pragma unroll
            for (int rr = 0; rr < kElocStage; ++rr) code[rr] = __builtin_amdgcn_readfirstlane(cv[rr]);
            constexpr int kStep = KE / kElocStage;           // staging slots every kStep fragments
            constexpr int kStageAt = PH ? kStep / 2 : 0;     // first staging slot
            const T *Hc = Hs + (size_t)(p & 1) * kElocRows * ldh + lr * ldh + 8 * lh;
            T *Hn = Hs + (size_t)((p + 1) & 1) * kElocRows * ldh;
            const int nbase = (p + 1) * kElocRows;
            mc_floatx16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
            frag b[3];
            b[0] = *reinterpret_cast<const frag *>(Hc);
            b[1] = *reinterpret_cast<const frag *>(Hc + 16);
#pragma unroll
            for (int kf = 0; kf < KE; ++kf) {
                if (kf + 2 < KE) b[(kf + 2) % 3] = *reinterpret_cast<const frag *>(Hc + (kf + 2) * 16);
                __builtin_amdgcn_sched_barrier(0);
                acc = Mc<T>::mma(a[kf], b[kf % 3], acc);
                __builtin_amdgcn_sched_barrier(0);
                if (kf >= kStageAt && (kf - kStageAt) % kStep == 0 && (kf - kStageAt) / kStep < kElocStage) {
                    const int rr = (kf - kStageAt) / kStep, r = wave * kElocStage + rr;
                    eloc_stage_row_code<T>(W1l, code[rr], rg, zs, Hn, ldh, K, nch, min(nbase + r, nrows - 1), r, lane);
                }
            }
            read_codes(p + 2, cv);
            float abs_sum = 0.0f, prod = 1.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) eloc_logcosh4(acc, q, b2v[2 * q], abs_sum, prod);
            finish_tile(abs_sum, prod, p);
        };
        constexpr bool kPhase = KE <= 26;                // wider layers: the shifted copy would spill registers
        for (int p = 0; p < npass; ++p) {
            if (p >= 1) row_sums(p - 1, nrows);          // its partials were written before the last barrier
            if (!live) stage_pass(p + 1);
            else if (kPhase && late_phase) pass(p, std::true_type{});
            else pass(p, std::false_type{});
            __syncthreads();
        }
        row_sums(npass - 1, nrows);
        __syncthreads();
        // wave s sums sample s:  eps = diag + sum_rows coef * exp(f_row - f_sample)   (FP64)
        if (wave < ns) {
            const int s = wave, rend = r0 + 1 + rcnt[s];
            const float f0 = fr[r0];
            double off = 0.0;
            for (int r = r0 + 1 + lane; r < rend; r += 64) off += (double)rc[r] * exp((double)(fr[r] - f0));
            off = group_sum<64>(off);
            if (lane == 0) A.eloc[g0 + s] = diag[s] + off;
        }
    }
}

}  // namespace nqs
