// Two-layer dense network on the matrix cores:
//   z1 = W1 s + b1,  h1 = ReLU(z1),  z2 = W2 h1 + b2,  log|psi| = sum_k log cosh(z2_k).
//
// A block of 256 threads (4 waves) evaluates 64 "rows" at a time (64 chains
// of the sampler, or 64 moves of one sample in the local energy).  Each row's
// first layer is updated incrementally from a kept z1 (a flip of site i adds
// -2 s_i W1[:,i]; an exchange of antiparallel i, j adds -2 s_i (W1[:,i] -
// W1[:,j])), passed through ReLU and rounded to the operand format into LDS.
// The second layer is one GEMM on the matrix cores, Z2^T = W2 H1^T, with W2
// streamed through L2 (A operand) and H1 from LDS (B operand), so that each
// lane's output fragment covers 16 outputs of ONE row: the log-cosh sum then
// needs no cross-lane work except one exchange between the two half-waves.
// log cosh is summed as  sum |z| + log prod (1 + e^{-2|z|}) - n log 2, one
// logarithm per 32 outputs.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace nqs {

typedef float mc_floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 mc_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 mc_halfx8 __attribute__((ext_vector_type(8)));

template <typename T>
struct Mc;

template <>
struct Mc<__bf16> {
    static constexpr int EPL = 8;   // K elements per lane per instruction (K = 16)
    typedef mc_bf16x8 frag;
    static __device__ __forceinline__ mc_floatx16 mma(frag a, frag b, mc_floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ __bf16 from_f32(float v) { return (__bf16)v; }
    static __device__ __forceinline__ float to_f32(__bf16 v) { return (float)v; }
};

template <>
struct Mc<_Float16> {
    static constexpr int EPL = 8;
    typedef mc_halfx8 frag;
    static __device__ __forceinline__ mc_floatx16 mma(frag a, frag b, mc_floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ _Float16 from_f32(float v) { return (_Float16)v; }
    static __device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
};

template <>
struct Mc<float> {
    static constexpr int EPL = 1;   // K = 2
    typedef float frag;
    static __device__ __forceinline__ mc_floatx16 mma(frag a, frag b, mc_floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ float from_f32(float v) { return v; }
    static __device__ __forceinline__ float to_f32(float v) { return v; }
};

constexpr int kRows = 64;        // rows evaluated per block pass
constexpr float kLn2f = 0.69314718055994531f;

template <typename T>
__host__ __device__ constexpr int hs_pad()
{
    return sizeof(T) == 2 ? 8 : 4;
}

// Layer 2 + log-cosh sum of the kRows staged rows Hs[kRows][ldh].  Writes
// part[wave][row] (LDS); the caller sums the 4 wave partials after a barrier.
// b2s: LDS copy of the padded bias.  W2: global [m2p][m1p] in T.
template <typename T>
__device__ __forceinline__ void gemm_logcosh_rows(const T *__restrict__ W2, const float *b2s, const T *Hs, int ldh,
                                                  int m1p, int m2p, float *part)
{
    typedef typename Mc<T>::frag frag;
    constexpr int EPL = Mc<T>::EPL;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    float abs_sum[2] = {0.0f, 0.0f}, prod[2] = {1.0f, 1.0f};
    int e2[2] = {0, 0};
    int nrow = 0;
    for (int rb = wave * 64; rb < m2p; rb += 256) {
        mc_floatx16 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
        const T *wrow0 = W2 + (size_t)(rb + lr) * m1p + lh * EPL;
        const T *wrow1 = W2 + (size_t)(rb + 32 + lr) * m1p + lh * EPL;
        const T *hrow0 = Hs + lr * ldh + lh * EPL;
        const T *hrow1 = Hs + (32 + lr) * ldh + lh * EPL;
        for (int k0 = 0; k0 < m1p; k0 += 2 * EPL) {
            const frag a0 = *reinterpret_cast<const frag *>(wrow0 + k0);
            const frag a1 = *reinterpret_cast<const frag *>(wrow1 + k0);
            const frag b0 = *reinterpret_cast<const frag *>(hrow0 + k0);
            const frag b1 = *reinterpret_cast<const frag *>(hrow1 + k0);
            acc[0][0] = Mc<T>::mma(a0, b0, acc[0][0]);
            acc[0][1] = Mc<T>::mma(a0, b1, acc[0][1]);
            acc[1][0] = Mc<T>::mma(a1, b0, acc[1][0]);
            acc[1][1] = Mc<T>::mma(a1, b1, acc[1][1]);
        }
        // D[i][j] of a 32x32 tile: lane = j + 32*((i/4)%2), register = i%4 + 4*(i/8).
        // Here i = output (row of W2), j = staged row.
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int out = rb + 32 * a + 8 * (r >> 2) + 4 * lh + (r & 3);
                const float bias = b2s[out];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const float v = fabsf(acc[a][b][r] + bias);
                    abs_sum[b] += v;
                    prod[b] *= 1.0f + __expf(-2.0f * v);
                }
            }
        nrow += 32;
#pragma unroll
        for (int b = 0; b < 2; ++b) {   // each factor is in (1, 2]: renormalise once per 32
            int e;
            prod[b] = frexpf(prod[b], &e);
            e2[b] += e;
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        float s = abs_sum[b] + __logf(prod[b]) + ((float)e2[b] - (float)nrow) * kLn2f;
        s += __shfl_xor(s, 32, 64);   // the other half-wave holds the other outputs of the same row
        if (lh == 0) part[wave * kRows + 32 * b + lr] = s;
    }
}

// ---------------------------------------------------------------------------
// Sampler
// ---------------------------------------------------------------------------
struct FfnnSampleArgs {
    FfnnDev net;
    const void *W2;    // [m2p][m1p] in the operand format
    const void *W1t;   // [N][m1p] in the operand format (layer-1 columns, LDS staged)
    int8_t *chain_state;
    int8_t *samples;
    float *logpsi;
    unsigned long long *n_acc;
    int64_t n_chains;
    int n_sweeps, n_burnin, sweep_size, refresh_sweeps;
    int move;          // 0 flip, 1 exchange
    uint64_t seed, step_offset;
    uint32_t inst, chain_id_offset;
    int n_traced;
    int32_t *tr_site;
    uint32_t *tr_ubits;
    float *tr_delta;
    uint8_t *tr_acc;
};

template <typename T>
struct FfnnLds {
    // carved from dynamic LDS in this order
    static __host__ __device__ size_t bytes(int N, int m1p, int m2p)
    {
        const size_t ldh = m1p + hs_pad<T>();
        const int NW = (N + 31) / 32;
        size_t b = 0;
        if (sizeof(T) == 2) b += sizeof(T) * (size_t)N * m1p;   // W1t (16-bit operands only)
        b += sizeof(T) * (size_t)kRows * ldh;                  // Hs
        b += sizeof(float) * m2p;                              // b2s
        b += sizeof(float) * 4 * kRows;                        // part
        b += sizeof(uint32_t) * (size_t)kRows * NW;            // spin words
        b += sizeof(int) * kRows * 4 + sizeof(float) * kRows * 3;   // proposal / state per row
        return b;
    }
};

template <typename T, int QK, bool TRACE>
__global__ void __launch_bounds__(256) ffnn_sample_kernel(FfnnSampleArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const FfnnDev &net = A.net;
    const int N = net.widths[0], m1p = net.m1p, m2p = net.m2p;
    const int NW = (N + 31) >> 5;
    const int ldh = m1p + hs_pad<T>();
    constexpr bool W1_LDS = sizeof(T) == 2;
    T *W1l = reinterpret_cast<T *>(smem);
    T *Hs = W1l + (W1_LDS ? (size_t)N * m1p : 0);
    const T *W1s = W1_LDS ? W1l : reinterpret_cast<const T *>(A.W1t);
    float *b2s = reinterpret_cast<float *>(Hs + (size_t)kRows * ldh);
    float *part = b2s + m2p;
    uint32_t *words = reinterpret_cast<uint32_t *>(part + 4 * kRows);
    int *pi = reinterpret_cast<int *>(words + kRows * NW);
    int *pj = pi + kRows;
    int *peff = pj + kRows;
    int *pupd = peff + kRows;
    float *pl2u = reinterpret_cast<float *>(pupd + kRows);
    float *fcur = pl2u + kRows;
    float *psgn = fcur + kRows;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kRows;
    const int nvalid = (int)min<int64_t>(kRows, A.n_chains - c0);

    // stage layer-1 columns and the bias, load spins
    {
        if constexpr (W1_LDS) {
            const T *src = reinterpret_cast<const T *>(A.W1t);
            const int n = N * m1p;
            for (int k = tid; k < n; k += 256) W1l[k] = src[k];
        }
        for (int k = tid; k < m2p; k += 256) b2s[k] = net.b2p[k];
        for (int k = tid; k < kRows * NW; k += 256) {
            const int r = k / NW, w = k % NW;
            uint32_t bits = 0;
            if (r < nvalid) {
                const int8_t *s = A.chain_state + (c0 + r) * N + 32 * w;
                const int nb = min(32, N - 32 * w);
                for (int b = 0; b < nb; ++b) bits |= (s[b] > 0 ? 1u : 0u) << b;
            }
            words[k] = bits;
        }
    }
    __syncthreads();

    // z1 of this wave's 16 rows: lane owns hidden units k = lane + 64 q
    constexpr int RPW = kRows / 4;
    float z1[RPW][QK];
    auto refresh_z1 = [&]() {
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int q = 0; q < QK; ++q) {
                const int k = lane + 64 * q;
                z1[r][q] = k < m1p ? net.b1p[k] : 0.0f;
            }
        for (int i = 0; i < N; ++i) {
            float w[QK];
#pragma unroll
            for (int q = 0; q < QK; ++q) {
                const int k = lane + 64 * q;
                w[q] = k < m1p ? Mc<T>::to_f32(W1s[i * m1p + k]) : 0.0f;
            }
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int row = wave * RPW + r;
                const float s = ((words[row * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1.0f : -1.0f;
#pragma unroll
                for (int q = 0; q < QK; ++q) z1[r][q] = fmaf(w[q], s, z1[r][q]);
            }
        }
    };
    // layer-1 change of row r's proposal, dz[q] (0 when the proposal changes nothing)
    auto delta_z1 = [&](int row, float (&dz)[QK]) {
        const int i = pi[row], j = pj[row];
        const float g = -2.0f * psgn[row];
#pragma unroll
        for (int q = 0; q < QK; ++q) {
            const int k = lane + 64 * q;
            float d = 0.0f;
            if (k < m1p && peff[row]) {
                d = Mc<T>::to_f32(W1s[i * m1p + k]);
                if (j >= 0) d -= Mc<T>::to_f32(W1s[j * m1p + k]);
            }
            dz[q] = g * d;
        }
    };
    // stage h1 = ReLU(z1 + dz) of this wave's rows (operand format)
    auto stage = [&](bool with_proposal) {
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = wave * RPW + r;
            float dz[QK];
            if (with_proposal) delta_z1(row, dz);
#pragma unroll
            for (int q = 0; q < QK; ++q) {
                const int k = lane + 64 * q;
                if (k < m1p) {
                    const float h = fmaxf(z1[r][q] + (with_proposal ? dz[q] : 0.0f), 0.0f);
                    Hs[row * ldh + k] = Mc<T>::from_f32(h);
                }
            }
        }
    };
    const T *W2 = reinterpret_cast<const T *>(A.W2);

    refresh_z1();
    stage(false);
    __syncthreads();
    gemm_logcosh_rows<T>(W2, b2s, Hs, ldh, m1p, m2p, part);
    __syncthreads();
    if (tid < kRows) fcur[tid] = part[tid] + part[kRows + tid] + part[2 * kRows + tid] + part[3 * kRows + tid];

    const int sw = A.sweep_size;
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * sw;
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    unsigned long long acc = 0;
    int in_sweep = 0, since_refresh = 0;
    int64_t sweep = 0;
    for (int64_t k = 0; k < total; ++k) {
        // proposals (one thread per row)
        if (tid < kRows) {
            const uint64_t step = A.step_offset + (uint64_t)k;
            const uint32_t gid = A.chain_id_offset + (uint32_t)(c0 + tid);
            const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, A.inst << 8, key0, key1);
            const int i = index_from_word(rb.r0, N);
            int j = -1;
            if (A.move == 1) {
                j = index_from_word(rb.r1, N - 1);
                j += (j >= i) ? 1 : 0;
            }
            const uint32_t *w = words + tid * NW;
            const bool si = (w[i >> 5] >> (i & 31)) & 1u;
            const bool eff = tid < nvalid && (j < 0 || si != (bool)((w[j >> 5] >> (j & 31)) & 1u));
            pi[tid] = i;
            pj[tid] = j;
            peff[tid] = eff ? 1 : 0;
            psgn[tid] = si ? 1.0f : -1.0f;
            const uint32_t ub = rb.r2 >> 8;
            pl2u[tid] = __builtin_amdgcn_logf((float)ub * 5.9604644775390625e-8f);
            pupd[tid] = (int)ub;   // u bits kept for the trace until the decision
        }
        __syncthreads();
        stage(true);
        __syncthreads();
        gemm_logcosh_rows<T>(W2, b2s, Hs, ldh, m1p, m2p, part);
        __syncthreads();
        if (tid < kRows) {
            const float fnew = part[tid] + part[kRows + tid] + part[2 * kRows + tid] + part[3 * kRows + tid];
            const bool eff = peff[tid] != 0;
            const float d2 = eff ? 2.0f * (fnew - fcur[tid]) / kLn2f : 0.0f;
            const bool accept = pl2u[tid] < d2;
            const uint32_t ub = (uint32_t)pupd[tid];
            if (tid < nvalid && accept) ++acc;
            const bool upd = accept && eff;
            if (upd) {
                uint32_t *w = words + tid * NW;
                const int i = pi[tid], j = pj[tid];
                w[i >> 5] ^= 1u << (i & 31);
                if (j >= 0) w[j >> 5] ^= 1u << (j & 31);
                fcur[tid] = fnew;
            }
            if constexpr (TRACE) {
                const int64_t c = c0 + tid;
                if (c < A.n_traced) {
                    const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                    A.tr_site[idx] = pi[tid] | ((pj[tid] < 0 ? 0xFFFF : pj[tid]) << 16);
                    A.tr_ubits[idx] = ub;
                    A.tr_delta[idx] = d2 * kLn2f;
                    A.tr_acc[idx] = accept ? 1 : 0;
                }
            }
            pupd[tid] = upd ? 1 : 0;
        }
        __syncthreads();
        // apply accepted moves to z1
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = wave * RPW + r;
            if (pupd[row]) {
                float dz[QK];
                delta_z1(row, dz);
#pragma unroll
                for (int q = 0; q < QK; ++q) z1[r][q] += dz[q];
            }
        }
        if (++in_sweep == sw) {
            in_sweep = 0;
            const int64_t out = sweep - A.n_burnin;
            if (++since_refresh == A.refresh_sweeps) {
                refresh_z1();
                since_refresh = 0;
            }
            if (out >= 0) {
                if (A.samples) {
                    for (int idx = tid; idx < nvalid * N; idx += 256) {
                        const int r = idx / N, i = idx % N;
                        A.samples[((size_t)out * A.n_chains + c0 + r) * N + i] =
                            ((words[r * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1 : -1;
                    }
                }
                if (A.logpsi && tid < nvalid) A.logpsi[(size_t)out * A.n_chains + c0 + tid] = fcur[tid];
            }
            ++sweep;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < nvalid * N; idx += 256) {
        const int r = idx / N, i = idx % N;
        A.chain_state[(c0 + r) * N + i] = ((words[r * NW + (i >> 5)] >> (i & 31)) & 1u) ? 1 : -1;
    }
    if (A.n_acc && tid < nvalid) A.n_acc[c0 + tid] = acc;
}

// ---------------------------------------------------------------------------
// Local energies: row 0 of a sample is the sample itself, the other rows are
// the configurations connected to it by the Hamiltonian (every single flip
// for the TFIM; every antiparallel bond swap for the Heisenberg model), each
// with its matrix element times the Marshall sign ratio.
//   eps(s) = diag(s) + sum_rows coef_row * exp(f_row - f_0)        (FP64 sum)
// ---------------------------------------------------------------------------
struct FfnnElocArgs {
    FfnnDev net;
    const void *W2;
    const void *W1t;
    const int8_t *samples;
    int64_t n;
    int kind, dim, L, pbc, marshall;
    double J, h;
    double *eloc;
};

__device__ __forceinline__ bool on_sub_a(int dim, int L, int i)
{
    return dim == 1 ? (i % 2 == 0) : (((i / L) + (i % L)) % 2 == 0);
}

template <typename T>
__host__ __device__ inline size_t ffnn_eloc_lds_bytes(int N, int m1p, int m2p)
{
    const size_t ldh = m1p + hs_pad<T>();
    size_t b = 0;
    if (sizeof(T) == 2) b += sizeof(T) * (size_t)N * m1p;
    b += sizeof(T) * (size_t)kRows * ldh;
    b += sizeof(float) * (m2p + 4 * kRows + m1p + N);
    b += (sizeof(int) * 2 + sizeof(float) * 2) * (size_t)(2 * N + 1);
    return b;
}

template <typename T, int QK>
__global__ void __launch_bounds__(256) ffnn_eloc_kernel(FfnnElocArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const FfnnDev &net = A.net;
    const int N = net.widths[0], m1p = net.m1p, m2p = net.m2p;
    const int ldh = m1p + hs_pad<T>();
    const int maxmoves = 2 * N + 1;
    constexpr bool W1_LDS = sizeof(T) == 2;
    T *W1l = reinterpret_cast<T *>(smem);
    T *Hs = W1l + (W1_LDS ? (size_t)N * m1p : 0);
    const T *W1s = W1_LDS ? W1l : reinterpret_cast<const T *>(A.W1t);
    float *b2s = reinterpret_cast<float *>(Hs + (size_t)kRows * ldh);
    float *part = b2s + m2p;
    float *zs = part + 4 * kRows;                      // [m1p] z1 of the sample
    float *sp = zs + m1p;                              // [N] spins
    int *mi = reinterpret_cast<int *>(sp + N);         // [maxmoves]
    int *mj = mi + maxmoves;
    float *mc = reinterpret_cast<float *>(mj + maxmoves);   // coefficients
    float *fr = mc + maxmoves;                         // f of each row
    __shared__ int s_nmoves;
    __shared__ int s_wcount[4];
    __shared__ double s_red[4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        if constexpr (W1_LDS) {
            const T *src = reinterpret_cast<const T *>(A.W1t);
            for (int k = tid; k < N * m1p; k += 256) W1l[k] = src[k];
        }
        for (int k = tid; k < m2p; k += 256) b2s[k] = net.b2p[k];
    }
    const T *W2 = reinterpret_cast<const T *>(A.W2);
    const int nb = A.dim == 1 ? (A.pbc ? A.L : A.L - 1) : 2 * A.L * A.L;   // candidate bonds (2D: 2 per site)
    for (int64_t smp = blockIdx.x; smp < A.n; smp += gridDim.x) {
        __syncthreads();
        for (int i = tid; i < N; i += 256) sp[i] = (float)A.samples[smp * N + i];
        __syncthreads();
        for (int k = tid; k < m1p; k += 256) {
            float z = net.b1p[k];
            for (int i = 0; i < N; ++i) z = fmaf(Mc<T>::to_f32(W1s[i * m1p + k]), sp[i], z);
            zs[k] = z;
        }
        // diagonal part and the list of connected configurations
        double diag = 0.0;
        if (tid == 0) {
            mi[0] = -1;
            mj[0] = -1;
            mc[0] = 0.0f;
        }
        int cnt = 0;   // per-wave compaction with ballots
        const int ncand = A.kind == NQS_TFIM ? N : nb;
        const int nloop = ncand > nb ? ncand : nb;
        for (int base = 0; base < nloop; base += 256) {
            const int c = base + tid;
            int i = -1, j = -1;
            bool take = false;
            float coef = 0.0f;
            if (c < ncand) {
                if (A.kind == NQS_TFIM) {
                    i = c;
                    take = true;
                    coef = (float)A.h * ((A.marshall && on_sub_a(A.dim, A.L, i)) ? -1.0f : 1.0f);
                }
                // bonds (both models contribute the diagonal J s_i s_j)
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
                    diag += A.J * (double)(sp[bi] * sp[bj]);
                    if (A.kind == NQS_HEISENBERG && sp[bi] != sp[bj]) {
                        i = bi;
                        j = bj;
                        take = true;
                        const bool flip = A.marshall && (on_sub_a(A.dim, A.L, bi) != on_sub_a(A.dim, A.L, bj));
                        coef = 2.0f * (float)A.J * (flip ? -1.0f : 1.0f);
                    }
                }
            }
            const unsigned long long bal = __ballot(take);
            if (lane == 0) s_wcount[wave] = __popcll(bal);
            __syncthreads();
            int off = 1 + cnt;
            for (int w = 0; w < wave; ++w) off += s_wcount[w];
            const int tot = s_wcount[0] + s_wcount[1] + s_wcount[2] + s_wcount[3];
            if (take) {
                const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
                mi[pos] = i;
                mj[pos] = j;
                mc[pos] = coef;
            }
            cnt += tot;
            __syncthreads();
        }
        const int nrows = 1 + cnt;
        // evaluate rows in passes of kRows
        for (int r0 = 0; r0 < nrows; r0 += kRows) {
            __syncthreads();
            for (int r = 0; r < kRows / 4; ++r) {
                const int row = r0 + wave * (kRows / 4) + r;
                const int lr = row - r0;
                int i = -1, j = -1;
                float g = 0.0f;
                if (row < nrows) {
                    i = mi[row];
                    j = mj[row];
                    g = i >= 0 ? -2.0f * sp[i] : 0.0f;
                }
#pragma unroll
                for (int q = 0; q < QK; ++q) {
                    const int k = lane + 64 * q;
                    if (k < m1p) {
                        float d = 0.0f;
                        if (i >= 0) {
                            d = Mc<T>::to_f32(W1s[i * m1p + k]);
                            if (j >= 0) d -= Mc<T>::to_f32(W1s[j * m1p + k]);
                        }
                        const float hv = fmaxf(fmaf(g, d, zs[k]), 0.0f);
                        Hs[lr * ldh + k] = Mc<T>::from_f32(hv);
                    }
                }
            }
            __syncthreads();
            gemm_logcosh_rows<T>(W2, b2s, Hs, ldh, m1p, m2p, part);
            __syncthreads();
            if (tid < kRows && r0 + tid < nrows)
                fr[r0 + tid] = part[tid] + part[kRows + tid] + part[2 * kRows + tid] + part[3 * kRows + tid];
        }
        __syncthreads();
        const float f0 = fr[0];
        double off = 0.0;
        for (int r = 1 + tid; r < nrows; r += 256) off += (double)mc[r] * exp((double)(fr[r] - f0));
        double v = group_sum<64>(diag + off);
        if (lane == 0) s_red[wave] = v;
        __syncthreads();
        if (tid == 0) A.eloc[smp] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    }
}

}  // namespace nqs
