// Two-layer dense network with layer 2 held in registers (16-bit operands).
//   z1 = W1 s + b1,  h1 = ReLU(z1),  z2 = W2 h1 + b2,  log|psi| = sum_k log cosh(z2_k).
//
// A block of 512 threads (8 waves) keeps W2 resident for its whole life: wave w
// holds output rows 32w .. 32w+31 of W2 as the A fragments of
// v_mfma_f32_32x32x16_{bf16,f16} (KF fragments of 8 values per lane, K = 16 per
// fragment).  The rows to evaluate are staged once per pass into LDS as the B
// operand (h1 rows, one row per matrix column), so the only per-pass traffic is
// LDS reads of h1; no weight is re-read from L2 inside the loop.  Each wave
// turns its 32 x 32 tile into per-row partial log-cosh sums over its 32
// outputs; the partials of the waves are added in wave order.
//
// Sampler: 64 chains per block; wave w keeps z1 of chains 8w .. 8w+7 in
// registers (lane owns hidden units lane + 64 q) and updates it by the rank-1
// (flip) or rank-2 (exchange) change of an accepted move.  Proposals that
// change nothing (an exchange of equal spins) are compacted away before the
// matrix product, so a pass evaluates only the effective proposals.
// Local energies: 4 samples per group; their connected configurations are
// listed, laid end to end and evaluated 32 rows per pass.
#pragma once

#include <hip/hip_runtime.h>

#include "ffnn_mc.h"

namespace nqs {

constexpr int kRegThreads = 512;
constexpr int kRegWaves = kRegThreads / 64;
constexpr int kRegRows = 64;       // chains per sampler block
constexpr int kRegPass = 32;       // rows per local-energy pass
constexpr int kRegGroup = 4;       // samples per local-energy group

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

// Rows row0 .. row0+31 of Hs (ldh elements per row) through layer 2 and the
// log-cosh sum over this wave's outputs; lanes 0..31 return the partial of
// row row0 + lane (other lanes return the same value for their row).
template <typename T, int KF>
__device__ __forceinline__ float reg_tile_logcosh(const typename Mc<T>::frag (&a)[KF], const T *Hs, int ldh, int row0,
                                                  const float *b2s, int m2)
{
    typedef typename Mc<T>::frag frag;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    // two accumulators (even / odd fragments), so consecutive matrix-core steps do not wait on each other
    mc_floatx16 acc, acc1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc[r] = 0.0f;
        acc1[r] = 0.0f;
    }
    const T *hrow = Hs + (row0 + lr) * ldh + 8 * lh;
#pragma unroll
    for (int kf = 0; kf < KF; kf += 2) {
        const frag b0 = *reinterpret_cast<const frag *>(hrow + kf * 16);
        acc = Mc<T>::mma(a[kf], b0, acc);
        if (kf + 1 < KF) {
            const frag b1 = *reinterpret_cast<const frag *>(hrow + (kf + 1) * 16);
            acc1 = Mc<T>::mma(a[kf + 1], b1, acc1);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += acc1[r];
    // D[i][j]: i = output (row of W2), j = staged row; lane = j + 32*((i/4)%2), register = i%4 + 4*(i/8)
    float abs_sum = 0.0f, prod = 1.0f;
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int out = wave * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        if (out < m2) {
            const float v = fabsf(acc[r] + b2s[out]);
            abs_sum += v;
            prod *= 1.0f + __expf(-2.0f * v);
            ++cnt;
        }
    }
    // 16 factors in (1, 2]: the product stays below 2^16
    float s = abs_sum + __logf(prod) - (float)cnt * kLn2f;
    s += __shfl_xor(s, 32, 64);
    return s;
}

// ---------------------------------------------------------------------------
// Sampler
// ---------------------------------------------------------------------------
template <typename T>
struct RegSampleLds {
    static __host__ __device__ size_t bytes(int N, int m1p, int m2p)
    {
        const size_t ldh = m1p + hs_pad<T>();
        const int NW = (N + 31) / 32;
        size_t b = 0;
        b += sizeof(T) * (size_t)N * m1p;                     // W1 columns
        b += sizeof(T) * (size_t)kRegRows * ldh;              // h1 rows
        b += sizeof(float) * m2p;                             // b2
        b += sizeof(float) * kRegWaves * kRegRows;            // partial sums
        b += sizeof(uint32_t) * (size_t)kRegRows * NW;        // spin words
        b += sizeof(int) * 4 + 16;                            // slot counters
        return b;
    }
};

// Each wave owns 8 chains: it draws their proposals (lanes 0..7), stages the
// effective ones at slots taken from a shared counter, and after the matrix
// product decides them and updates their state.  Two barriers per step: after
// the staging (h1 rows complete) and after the product (partial sums complete).
template <typename T, int KF, bool TRACE>
__global__ void __launch_bounds__(kRegThreads) ffnn_sample_reg_kernel(FfnnSampleArgs A)
{
    typedef typename Mc<T>::frag frag;
    constexpr int QK = KF / 4;                      // hidden units per lane (m1p = 64 QK)
    constexpr int RPW = kRegRows / kRegWaves;       // chains per wave (8)
    extern __shared__ __align__(16) unsigned char smem[];
    const FfnnDev &net = A.net;
    const int N = net.widths[0], m1p = net.m1p, m2p = net.m2p, m2 = net.widths[2];
    const int NW = (N + 31) >> 5;
    const int ldh = m1p + hs_pad<T>();
    const int nwt = (m2p + 31) >> 5;                // waves that own output rows
    T *W1l = reinterpret_cast<T *>(smem);
    T *Hs = W1l + (size_t)N * m1p;
    float *b2s = reinterpret_cast<float *>(Hs + (size_t)kRegRows * ldh);
    float *part = b2s + m2p;
    uint32_t *words = reinterpret_cast<uint32_t *>(part + kRegWaves * kRegRows);
    int *cnt = reinterpret_cast<int *>(words + kRegRows * NW);   // [2] slots taken in the current / next step

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kRegRows;
    const int nvalid = (int)min<int64_t>(kRegRows, A.n_chains - c0);
    const int myrow = wave * RPW + (lane & (RPW - 1));           // the chain of proposal lanes 0..7
    const bool plane = lane < RPW && myrow < nvalid;

    frag a[KF];
    reg_load_w2<T, KF>(reinterpret_cast<const T *>(A.W2), m1p, m2p, a);
    {
        const T *src = reinterpret_cast<const T *>(A.W1t);
        for (int k = tid; k < N * m1p; k += kRegThreads) W1l[k] = src[k];
        for (int k = tid; k < kRegRows * ldh; k += kRegThreads) Hs[k] = Mc<T>::from_f32(0.0f);
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
        if (tid < 2) cnt[tid] = 0;
    }
    __syncthreads();

    float z1[RPW][QK];
    auto refresh_z1 = [&]() {
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int q = 0; q < QK; ++q) z1[r][q] = net.b1p[lane + 64 * q];
        for (int i = 0; i < N; ++i) {
            float w[QK];
#pragma unroll
            for (int q = 0; q < QK; ++q) w[q] = Mc<T>::to_f32(W1l[i * m1p + lane + 64 * q]);
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int row = wave * RPW + r;
                const float s = ((words[row * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1.0f : -1.0f;
#pragma unroll
                for (int q = 0; q < QK; ++q) z1[r][q] = fmaf(w[q], s, z1[r][q]);
            }
        }
    };
    // layer-1 change of flipping i (and j >= 0) where site i holds spin si
    auto delta_z1 = [&](int i, int j, float si, float (&dz)[QK]) {
        const float g = -2.0f * si;
#pragma unroll
        for (int q = 0; q < QK; ++q) {
            const int k = lane + 64 * q;
            float d = Mc<T>::to_f32(W1l[i * m1p + k]);
            if (j >= 0) d -= Mc<T>::to_f32(W1l[j * m1p + k]);
            dz[q] = g * d;
        }
    };
    // log|psi| of this wave's chains from the current z1 (lanes 0..7 return their chain's value)
    auto full_eval = [&]() -> float {
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = wave * RPW + r;
#pragma unroll
            for (int q = 0; q < QK; ++q) Hs[row * ldh + lane + 64 * q] = Mc<T>::from_f32(fmaxf(z1[r][q], 0.0f));
        }
        __syncthreads();
        for (int t = 0; t < kRegRows / 32; ++t) {
            const float s = reg_tile_logcosh<T, KF>(a, Hs, ldh, 32 * t, b2s, m2);
            if (lane < 32) part[wave * kRegRows + 32 * t + lane] = s;
        }
        __syncthreads();
        float f = 0.0f;
        for (int w = 0; w < nwt; ++w) f += part[w * kRegRows + myrow];
        return f;
    };

    refresh_z1();
    float fcur = full_eval();   // meaningful on proposal lanes

    const int sw = A.sweep_size;
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * sw;
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    unsigned long long acc = 0;
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
        // stage h1 of the effective proposals (rows are wave-uniform)
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int sl = __builtin_amdgcn_readlane(slot, r);
            if (sl >= 0) {
                const int i = __builtin_amdgcn_readlane(pi, r), j = __builtin_amdgcn_readlane(pj, r);
                const float s_i = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(si), r));
                float dz[QK];
                delta_z1(i, j, s_i, dz);
#pragma unroll
                for (int q = 0; q < QK; ++q)
                    Hs[sl * ldh + lane + 64 * q] = Mc<T>::from_f32(fmaxf(z1[r][q] + dz[q], 0.0f));
            }
        }
        __syncthreads();
        const int neff = cnt[k & 1];
        for (int t = 0; 32 * t < neff; ++t) {
            const float s = reg_tile_logcosh<T, KF>(a, Hs, ldh, 32 * t, b2s, m2);
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
                float dz[QK];
                delta_z1(i, j, s_i, dz);
#pragma unroll
                for (int q = 0; q < QK; ++q) z1[r][q] += dz[q];
            }
        }
        if (++in_sweep == sw) {
            in_sweep = 0;
            const int64_t out = sweep - A.n_burnin;
            if (++since_refresh == A.refresh_sweeps) {
                refresh_z1();
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
    for (int idx = lane; idx < RPW * N; idx += 64) {
        const int r = idx / N, i = idx % N, row = wave * RPW + r;
        if (row < nvalid)
            A.chain_state[(c0 + row) * N + i] = ((words[row * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1 : -1;
    }
    if (A.n_acc && plane) A.n_acc[c0 + myrow] = acc;
}

// ---------------------------------------------------------------------------
// Local energies
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ inline size_t reg_eloc_lds_bytes(int N, int m1p, int m2p)
{
    const size_t ldh = m1p + hs_pad<T>();
    const size_t maxrows = (size_t)kRegGroup * (2 * N + 1);
    size_t b = 0;
    b += sizeof(T) * (size_t)N * m1p;                   // W1 columns
    b += sizeof(T) * (size_t)kRegPass * ldh;            // h1 rows of a pass
    b += sizeof(float) * m2p;                           // b2
    b += sizeof(float) * kRegWaves * kRegPass;          // partial sums
    b += sizeof(float) * (size_t)kRegGroup * m1p;       // z1 of the group's samples
    b += sizeof(float) * (size_t)kRegGroup * N;         // spins
    b += (sizeof(int) * 3 + sizeof(float) * 2) * maxrows;   // rows: site i, site j, sample, coefficient, f
    b += sizeof(double) * (kRegGroup + kRegWaves) + sizeof(int) * (kRegGroup + 2 + kRegWaves) + 16;
    return b;
}

template <typename T, int KF>
__global__ void __launch_bounds__(kRegThreads) ffnn_eloc_reg_kernel(FfnnElocArgs A)
{
    typedef typename Mc<T>::frag frag;
    constexpr int G = kRegGroup;
    extern __shared__ __align__(16) unsigned char smem[];
    const FfnnDev &net = A.net;
    const int N = net.widths[0], m1p = net.m1p, m2p = net.m2p, m2 = net.widths[2];
    const int ldh = m1p + hs_pad<T>();
    const int nwt = (m2p + 31) >> 5;
    const int maxrows = G * (2 * N + 1);
    T *W1l = reinterpret_cast<T *>(smem);
    T *Hs = W1l + (size_t)N * m1p;
    float *b2s = reinterpret_cast<float *>(Hs + (size_t)kRegPass * ldh);
    float *part = b2s + m2p;
    float *zs = part + kRegWaves * kRegPass;           // [G][m1p]
    float *sp = zs + (size_t)G * m1p;                  // [G][N]
    int *ri = reinterpret_cast<int *>(sp + (size_t)G * N);
    int *rj = ri + maxrows;
    int *rs = rj + maxrows;
    float *rc = reinterpret_cast<float *>(rs + maxrows);
    float *fr = rc + maxrows;
    double *diag = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(fr + maxrows) + 7) & ~(uintptr_t)7);
    double *dred = diag + G;                           // [kRegWaves]
    int *rbase = reinterpret_cast<int *>(dred + kRegWaves);   // [G] first row of each sample
    int *s_nrows = rbase + G;
    int *wcount = s_nrows + 2;                         // [kRegWaves]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    frag a[KF];
    reg_load_w2<T, KF>(reinterpret_cast<const T *>(A.W2), m1p, m2p, a);
    {
        const T *src = reinterpret_cast<const T *>(A.W1t);
        for (int k = tid; k < N * m1p; k += kRegThreads) W1l[k] = src[k];
        for (int k = tid; k < kRegPass * ldh; k += kRegThreads) Hs[k] = Mc<T>::from_f32(0.0f);
        for (int k = tid; k < m2p; k += kRegThreads) b2s[k] = net.b2p[k];
    }
    const int nb = A.dim == 1 ? (A.pbc ? A.L : A.L - 1) : 2 * A.L * A.L;   // candidate bonds (2D: 2 per site)
    const int ncand = A.kind == NQS_TFIM ? N : 0;
    const int nloop = ncand > nb ? ncand : nb;

    for (int64_t g0 = (int64_t)blockIdx.x * G; g0 < A.n; g0 += (int64_t)gridDim.x * G) {
        const int ns = (int)min<int64_t>(G, A.n - g0);
        __syncthreads();
        for (int k = tid; k < G * N; k += kRegThreads) {
            const int s = k / N, i = k % N;
            sp[k] = s < ns ? (float)A.samples[(g0 + s) * N + i] : 1.0f;
        }
        if (tid == 0) *s_nrows = 0;
        __syncthreads();
        // z1 of the group's samples
        for (int k = tid; k < G * m1p; k += kRegThreads) {
            const int s = k / m1p, kk = k % m1p;
            float z = net.b1p[kk];
            for (int i = 0; i < N; ++i) z = fmaf(Mc<T>::to_f32(W1l[i * m1p + kk]), sp[s * N + i], z);
            zs[k] = z;
        }
        // diagonal part and the rows: the sample itself, then its connected configurations
        for (int s = 0; s < ns; ++s) {
            const float *ss = sp + s * N;
            double dg = 0.0;
            int cnt = 0;
            if (tid == 0) {
                const int r0 = *s_nrows;
                rbase[s] = r0;
                ri[r0] = -1;
                rj[r0] = -1;
                rs[r0] = s;
                rc[r0] = 0.0f;
            }
            __syncthreads();
            const int first = *s_nrows + 1;
            for (int base = 0; base < nloop; base += kRegThreads) {
                const int c = base + tid;
                int i = -1, j = -1;
                bool take = false;
                float coef = 0.0f;
                if (c < ncand) {
                    i = c;
                    take = true;
                    coef = (float)A.h * ((A.marshall && on_sub_a(A.dim, A.L, i)) ? -1.0f : 1.0f);
                }
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
                    if (valid) {
                        dg += A.J * (double)(ss[bi] * ss[bj]);
                        if (A.kind == NQS_HEISENBERG && ss[bi] != ss[bj]) {
                            i = bi;
                            j = bj;
                            take = true;
                            const bool flip = A.marshall && (on_sub_a(A.dim, A.L, bi) != on_sub_a(A.dim, A.L, bj));
                            coef = 2.0f * (float)A.J * (flip ? -1.0f : 1.0f);
                        }
                    }
                }
                const unsigned long long bal = __ballot(take);
                if (lane == 0) wcount[wave] = __popcll(bal);
                __syncthreads();
                int off = first + cnt;
                for (int w = 0; w < wave; ++w) off += wcount[w];
                int tot = 0;
                for (int w = 0; w < kRegWaves; ++w) tot += wcount[w];
                if (take) {
                    const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
                    ri[pos] = i;
                    rj[pos] = j;
                    rs[pos] = s;
                    rc[pos] = coef;
                }
                cnt += tot;
                __syncthreads();
            }
            const double v = group_sum<64>(dg);
            if (lane == 0) dred[wave] = v;
            __syncthreads();
            if (tid == 0) {
                double d = 0.0;
                for (int w = 0; w < kRegWaves; ++w) d += dred[w];
                diag[s] = d;
                *s_nrows = first + cnt;
            }
            __syncthreads();
        }
        const int nrows = *s_nrows;
        // all rows through the network, kRegPass at a time
        for (int r0 = 0; r0 < nrows; r0 += kRegPass) {
            for (int rr = 0; rr < kRegPass / kRegWaves; ++rr) {
                const int lr = wave * (kRegPass / kRegWaves) + rr;
                const int row = r0 + lr;
                if (row < nrows) {
                    const int i = ri[row], j = rj[row], s = rs[row];
                    const float g = i >= 0 ? -2.0f * sp[s * N + i] : 0.0f;
                    for (int k = lane; k < m1p; k += 64) {
                        float d = 0.0f;
                        if (i >= 0) {
                            d = Mc<T>::to_f32(W1l[i * m1p + k]);
                            if (j >= 0) d -= Mc<T>::to_f32(W1l[j * m1p + k]);
                        }
                        Hs[lr * ldh + k] = Mc<T>::from_f32(fmaxf(fmaf(g, d, zs[s * m1p + k]), 0.0f));
                    }
                }
            }
            __syncthreads();
            const float sv = reg_tile_logcosh<T, KF>(a, Hs, ldh, 0, b2s, m2);
            if (lane < 32) part[wave * kRegPass + lane] = sv;
            __syncthreads();
            if (tid < kRegPass && r0 + tid < nrows) {
                float f = 0.0f;
                for (int w = 0; w < nwt; ++w) f += part[w * kRegPass + tid];
                fr[r0 + tid] = f;
            }
        }
        __syncthreads();
        // wave s sums sample s:  eps = diag + sum_rows coef * exp(f_row - f_sample)   (FP64)
        if (wave < ns) {
            const int s = wave, rb0 = rbase[s], rend = s + 1 < ns ? rbase[s + 1] : nrows;
            const float f0 = fr[rb0];
            double off = 0.0;
            for (int r = rb0 + 1 + lane; r < rend; r += 64) off += (double)rc[r] * exp((double)(fr[r] - f0));
            off = group_sum<64>(off);
            if (lane == 0) A.eloc[g0 + s] = diag[s] + off;
        }
    }
}

}  // namespace nqs
