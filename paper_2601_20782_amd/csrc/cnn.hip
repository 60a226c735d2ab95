// Residual convolutional network (App. H) on an L x L periodic lattice:
//   h0 = Conv(s);  h <- h + Conv(phi(Conv(phi(LN(h)))))  (R blocks);
//   log psi = sum over sites and channels of LN(h).
// Conv: 3 x 3 cross-correlation with circular padding and a bias per output
// channel; LN: per site over the F channels, learnable scale and shift,
// epsilon 1e-6; phi: GELU, tanh form.  Reduced precision: the parameters are
// rounded to the sampling format, and so is the input of every convolution
// after the first; sums, LN, GELU and the residual stream are FP32.
//
// Every evaluation is one configuration per workgroup, activations in LDS
// ([site][channel], FP32), weights read from the copy ([in channel][offset]
// [out channel], so consecutive threads (out channels) read consecutive words).
// The sampler runs one chain per workgroup (proposal, forward pass, decision);
// the local energy one sample per workgroup (the sample and its N flips).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "internal.h"

namespace nqs {

constexpr int kCnnThreads = 256;
constexpr float kLnEps = 1e-6f;

int64_t cnn_num_params(int F, int R)
{
    return 10 * (int64_t)F + (int64_t)R * (2 * F + 2 * (9 * (int64_t)F * F + F)) + 2 * (int64_t)F;
}

// ---- copy: round the FP64 master, rearrange each convolution's weights ----

struct CnnSeg {
    int64_t start, len;
    int conv;   // 0: copied as is; else a convolution with `conv` input channels: [o][c][k] -> [c][k][o]
    int F;
};

__global__ void cnn_build_kernel(const double *__restrict__ master, int64_t P, int dtype, const CnnSeg *__restrict__ segs,
                                 int nseg, float *__restrict__ out)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    int s = 0;
    while (s + 1 < nseg && q >= segs[s + 1].start) ++s;
    const CnnSeg g = segs[s];
    const float v = (float)round_to_dtype(master[q], dtype);
    const int64_t r = q - g.start;
    if (g.conv == 0) {
        out[q] = v;
    } else {
        const int C = g.conv, F = g.F;
        const int64_t o = r / (9 * C), rem = r - o * 9 * C, c = rem / 9, k = rem - c * 9;
        out[g.start + (c * 9 + k) * F + o] = v;
    }
}

// [offset][out][in] operands of the matrix-core convolutions from the rearranged
// FP32 values ([in][offset][out]); the values are exact in the copy's format.
__global__ void cnn_build_mc_kernel(CnnDev n, int64_t total)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int F = n.F;
    const int64_t per = 9 * (int64_t)F * F;
    const int rj = (int)(q / per);
    const int64_t e = q - rj * per;
    const int k = (int)(e / ((int64_t)F * F)), o = (int)((e / F) % F), c = (int)(e % F);
    const int r = rj >> 1;
    const float *W = n.p + ((rj & 1) ? n.w2[r] : n.w1[r]);
    const float v = W[((int64_t)c * 9 + k) * F + o];
    if (n.dtype == kF32) {
        reinterpret_cast<float *>(n.wmc)[q] = v;
    } else if (n.dtype == kBF16) {
        reinterpret_cast<uint16_t *>(n.wmc)[q] = (uint16_t)(__float_as_uint(v) >> 16);
    } else {
        const _Float16 hv = (_Float16)v;
        reinterpret_cast<uint16_t *>(n.wmc)[q] = *reinterpret_cast<const uint16_t *>(&hv);
    }
}

nqs_status cnn_build_copy(nqs_model *m, int dtype, hipStream_t stream)
{
    const nqs_model_desc &d = m->desc;
    if (dtype == NQS_FP8_E4M3) return set_error(NQS_EUNSUPPORTED, "FP8 copies of the convolutional network are not built");
    Copy &c = m->copies[dtype];
    CnnDev &n = c.cnn;
    n.L = d.lat_L;
    n.F = d.widths[0];
    n.R = d.n_layers;
    n.dtype = dtype;
    const int F = n.F;
    CnnSeg segs[8 * NQS_MAX_LAYERS + 8];
    int ns = 0;
    int64_t off = 0;
    auto seg = [&](int64_t len, int conv) {
        segs[ns++] = CnnSeg{off, len, conv, F};
        const int64_t at = off;
        off += len;
        return at;
    };
    n.w0 = seg(9 * (int64_t)F, 1);
    n.b0 = seg(F, 0);
    for (int r = 0; r < n.R; ++r) {
        n.g[r] = seg(F, 0);
        n.be[r] = seg(F, 0);
        n.w1[r] = seg(9 * (int64_t)F * F, F);
        n.b1[r] = seg(F, 0);
        n.w2[r] = seg(9 * (int64_t)F * F, F);
        n.b2[r] = seg(F, 0);
    }
    n.gf = seg(F, 0);
    n.bef = seg(F, 0);
    if (off != m->P) return set_error(NQS_EINVAL, "convolutional network parameter count mismatch");
    const size_t pbytes = (sizeof(float) * (size_t)m->P + 255) & ~(size_t)255;
    const size_t esz = dtype == NQS_F32 ? sizeof(float) : sizeof(uint16_t);
    const int64_t nmc = 2 * (int64_t)n.R * 9 * F * F;
    const size_t mcbytes = (esz * (size_t)nmc + 255) & ~(size_t)255;
    const size_t sbytes = (sizeof(segs) + 255) & ~(size_t)255;
    if (!c.block) NQS_HIP_TRY(hipMalloc(&c.block, pbytes + sbytes + mcbytes));
    n.p = (float *)c.block;
    CnnSeg *dsegs = (CnnSeg *)((char *)c.block + pbytes);
    n.wmc = (char *)c.block + pbytes + sbytes;
    NQS_HIP_TRY(hipMemcpyAsync(dsegs, segs, sizeof(CnnSeg) * ns, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(cnn_build_kernel, dim3((unsigned)((m->P + 255) / 256)), dim3(256), 0, stream, m->master, m->P,
                       dtype, dsegs, ns, n.p);
    NQS_HIP_TRY(hipGetLastError());
    if (nmc > 0) {
        hipLaunchKernelGGL(cnn_build_mc_kernel, dim3((unsigned)((nmc + 255) / 256)), dim3(256), 0, stream, n, nmc);
        NQS_HIP_TRY(hipGetLastError());
    }
    // the host array of segments must outlive the copy
    NQS_HIP_TRY(hipStreamSynchronize(stream));
    c.valid = true;
    return NQS_OK;
}

// ---- the forward pass of one configuration by one workgroup ----

struct CnnLds {
    float *x;     // [S] spins
    float *h;     // [S][F] residual stream
    float *t;     // [S][F] phi(LN(h)), rounded
    float *u;     // [S][F] phi(conv1), rounded
    float *red;   // [kCnnThreads / 64]
};

__host__ __device__ inline size_t cnn_lds_bytes(int S, int F)
{
    return sizeof(float) * ((size_t)S + 3 * (size_t)S * F + kCnnThreads / 64);
}

__device__ inline CnnLds cnn_carve(float *sm, int S, int F)
{
    CnnLds l;
    l.x = sm;
    l.h = sm + S;
    l.t = l.h + (size_t)S * F;
    l.u = l.t + (size_t)S * F;
    l.red = l.u + (size_t)S * F;
    return l;
}

__device__ inline int cnn_nbr(int s, int k, int L)
{
    const int x = s / L, y = s - (s / L) * L;
    int xx = x + k / 3 - 1, yy = y + k % 3 - 1;
    xx += xx < 0 ? L : (xx >= L ? -L : 0);
    yy += yy < 0 ? L : (yy >= L ? -L : 0);
    return xx * L + yy;
}

__device__ inline float cnn_gelu(float x)
{
    const float c = 0.7978845608028654f;   // sqrt(2 / pi)
    return 0.5f * x * (1.0f + tanhf(c * fmaf(0.044715f * x * x, x, x)));
}

// FP32 -> format -> FP32, round to nearest even: BF16 by rounding the low 16
// bits of the encoding (same exponent range; NaN kept quiet), FP16 by the
// hardware conversion (round to nearest even, overflow to infinity).
__device__ inline float cnn_round(float v, int dtype)
{
    if (dtype == kBF16) {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return __uint_as_float(u | 0x00400000u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return __uint_as_float(u & 0xffff0000u);
    }
    if (dtype == kF16) return (float)(_Float16)v;
    return v;
}

// out[s][o] (+)= b[o] + sum_{k, c} W[c][k][o] in[nbr(s, k)][c]
__device__ inline float cnn_conv_at(const float *__restrict__ W, const float *__restrict__ b, const float *in, int s,
                                    int o, int L, int C, int F)
{
    float acc = b[o];
    for (int k = 0; k < 9; ++k) {
        const float *src = in + (size_t)cnn_nbr(s, k, L) * C;
        const float *w = W + (size_t)k * F + o;
        for (int c = 0; c < C; ++c) acc = fmaf(w[(size_t)c * 9 * F], src[c], acc);
    }
    return acc;
}

// log psi of the configuration in l.x (all threads return it); ends with a barrier
__device__ float cnn_forward(const CnnDev &net, const CnnLds &l)
{
    const int L = net.L, S = L * L, F = net.F, tid = threadIdx.x;
    const float *P = net.p;
    for (int idx = tid; idx < S * F; idx += kCnnThreads) {
        const int s = idx / F, o = idx - (idx / F) * F;
        l.h[idx] = cnn_conv_at(P + net.w0, P + net.b0, l.x, s, o, L, 1, F);
    }
    __syncthreads();
    for (int r = 0; r < net.R; ++r) {
        const float *g = P + net.g[r], *be = P + net.be[r];
        for (int s = tid; s < S; s += kCnnThreads) {
            const float *hs = l.h + (size_t)s * F;
            float mu = 0.0f;
            for (int c = 0; c < F; ++c) mu += hs[c];
            mu /= (float)F;
            float var = 0.0f;
            for (int c = 0; c < F; ++c) var = fmaf(hs[c] - mu, hs[c] - mu, var);
            const float rs = 1.0f / sqrtf(var / (float)F + kLnEps);
            for (int c = 0; c < F; ++c)
                l.t[(size_t)s * F + c] = cnn_round(cnn_gelu(fmaf((hs[c] - mu) * rs, g[c], be[c])), net.dtype);
        }
        __syncthreads();
        for (int idx = tid; idx < S * F; idx += kCnnThreads) {
            const int s = idx / F, o = idx - (idx / F) * F;
            l.u[idx] = cnn_round(cnn_gelu(cnn_conv_at(P + net.w1[r], P + net.b1[r], l.t, s, o, L, F, F)), net.dtype);
        }
        __syncthreads();
        for (int idx = tid; idx < S * F; idx += kCnnThreads) {
            const int s = idx / F, o = idx - (idx / F) * F;
            l.h[idx] += cnn_conv_at(P + net.w2[r], P + net.b2[r], l.u, s, o, L, F, F);
        }
        __syncthreads();
    }
    const float *g = P + net.gf, *be = P + net.bef;
    float part = 0.0f;
    for (int s = tid; s < S; s += kCnnThreads) {
        const float *hs = l.h + (size_t)s * F;
        float mu = 0.0f;
        for (int c = 0; c < F; ++c) mu += hs[c];
        mu /= (float)F;
        float var = 0.0f;
        for (int c = 0; c < F; ++c) var = fmaf(hs[c] - mu, hs[c] - mu, var);
        const float rs = 1.0f / sqrtf(var / (float)F + kLnEps);
        for (int c = 0; c < F; ++c) part += fmaf((hs[c] - mu) * rs, g[c], be[c]);
    }
    part = group_sum<64>(part);
    if ((tid & 63) == 0) l.red[tid >> 6] = part;
    __syncthreads();
    float f = 0.0f;
    for (int w = 0; w < kCnnThreads / 64; ++w) f += l.red[w];
    __syncthreads();
    return f;
}

// ---- log psi of given configurations ----

__global__ void __launch_bounds__(kCnnThreads) cnn_logpsi_kernel(CnnDev net, const int8_t *__restrict__ samples,
                                                                 int64_t n, float *__restrict__ logpsi)
{
    extern __shared__ float sm[];
    const int S = net.L * net.L;
    const CnnLds l = cnn_carve(sm, S, net.F);
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        for (int i = threadIdx.x; i < S; i += kCnnThreads) l.x[i] = (float)samples[k * S + i];
        __syncthreads();
        const float f = cnn_forward(net, l);
        if (threadIdx.x == 0) logpsi[k] = f;
    }
}

// ---- Metropolis-Hastings, single flips, one chain per workgroup ----

struct CnnSampleArgs {
    CnnDev net;
    int8_t *chain_state;
    int8_t *samples;
    float *logpsi;
    unsigned long long *n_acc;
    int64_t n_chains;
    int n_sweeps, n_burnin, sweep_size;
    uint64_t seed, step_offset;
    uint32_t inst, chain_id_offset;
    int n_traced;
    int32_t *tr_site;
    uint32_t *tr_ubits;
    float *tr_delta;
    uint8_t *tr_acc;
};

__global__ void __launch_bounds__(kCnnThreads) cnn_sample_kernel(CnnSampleArgs A)
{
    extern __shared__ float sm[];
    __shared__ int s_site;
    __shared__ int s_accept;
    const int S = A.net.L * A.net.L, tid = threadIdx.x;
    const CnnLds l = cnn_carve(sm, S, A.net.F);
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * A.sweep_size;
    for (int64_t c = blockIdx.x; c < A.n_chains; c += gridDim.x) {
        const uint32_t gid = A.chain_id_offset + (uint32_t)c;
        for (int i = tid; i < S; i += kCnnThreads) l.x[i] = (float)A.chain_state[c * S + i];
        __syncthreads();
        float f = cnn_forward(A.net, l);
        unsigned long long acc = 0;
        for (int64_t k = 0; k < total; ++k) {
            const uint64_t step = A.step_offset + (uint64_t)k;
            uint32_t ub = 0;
            if (tid == 0) {
                const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, A.inst << 8, key0, key1);
                s_site = index_from_word(rb.r0, S);
                ub = rb.r2 >> 8;
                l.x[s_site] = -l.x[s_site];
            }
            __syncthreads();
            const float fn = cnn_forward(A.net, l);
            if (tid == 0) {
                const float d = 2.0f * (fn - f);
                const float l2u = __builtin_amdgcn_logf((float)ub * 5.9604644775390625e-8f);   // log2 u
                const bool accept = l2u < d * 1.4426950408889634f;                            // NaN rejects
                s_accept = accept ? 1 : 0;
                if (!accept) l.x[s_site] = -l.x[s_site];
                if (c < A.n_traced) {
                    const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                    A.tr_site[idx] = s_site | (0xFFFF << 16);
                    A.tr_ubits[idx] = ub;
                    A.tr_delta[idx] = d;
                    A.tr_acc[idx] = accept ? 1 : 0;
                }
            }
            __syncthreads();
            if (s_accept) {
                f = fn;
                ++acc;
            }
            if ((k + 1) % A.sweep_size == 0) {
                const int64_t out = (k + 1) / A.sweep_size - 1 - A.n_burnin;
                if (out >= 0) {
                    if (A.samples)
                        for (int i = tid; i < S; i += kCnnThreads)
                            A.samples[((size_t)out * A.n_chains + c) * S + i] = l.x[i] > 0.0f ? 1 : -1;
                    if (A.logpsi && tid == 0) A.logpsi[(size_t)out * A.n_chains + c] = f;
                    __syncthreads();   // the next proposal modifies l.x
                }
            }
        }
        for (int i = tid; i < S; i += kCnnThreads) A.chain_state[c * S + i] = l.x[i] > 0.0f ? 1 : -1;
        if (A.n_acc && tid == 0) A.n_acc[c] = acc;
        __syncthreads();
    }
}

// ---- TFIM local energies on the network's lattice, one sample per workgroup ----

__global__ void __launch_bounds__(kCnnThreads) cnn_eloc_tfim_kernel(CnnDev net, const int8_t *__restrict__ samples,
                                                                    int64_t n, double J, double h,
                                                                    double *__restrict__ eloc)
{
    extern __shared__ float sm[];
    const int L = net.L, S = L * L, tid = threadIdx.x;
    const CnnLds l = cnn_carve(sm, S, net.F);
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        for (int i = tid; i < S; i += kCnnThreads) l.x[i] = (float)samples[k * S + i];
        __syncthreads();
        const float f0 = cnn_forward(net, l);
        double off = 0.0;
        for (int i = 0; i < S; ++i) {
            if (tid == 0) l.x[i] = -l.x[i];
            __syncthreads();
            const float fi = cnn_forward(net, l);
            off += exp((double)(fi - f0));
            if (tid == 0) l.x[i] = -l.x[i];
            __syncthreads();
        }
        if (tid == 0) {
            double diag = 0.0;
            for (int s = 0; s < S; ++s) {
                const int x = s / L, y = s - (s / L) * L;
                const int right = ((x + 1) % L) * L + y, down = x * L + (y + 1) % L;
                diag += (double)(l.x[s] * l.x[right]) + (double)(l.x[s] * l.x[down]);
            }
            eloc[k] = J * diag + h * off;
        }
        __syncthreads();
    }
}

// ---- sampler with the convolutions on the matrix cores, B chains per workgroup ----
//
// The B chains of a workgroup propose in lockstep; the forward pass of their B
// proposed configurations is one batch: each convolution is a product of the
// [B*S rows][9 F] im2col matrix (gathered from LDS, the input of the
// convolution stored in the copy's format) with the [9 F][F] weights, in
// 16 x 16 tiles (v_mfma_f32_16x16x32_bf16 / _f16, 32 of the 9 F products per
// step, or v_mfma_f32_16x16x4_f32), FP32 accumulation; layer
// norms, GELU, biases and the residual stream stay FP32 as in the one-chain
// kernel.  Only the order of the FP32 sums differs from it.

typedef __bf16 cnn_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 cnn_h16x8 __attribute__((ext_vector_type(8)));
typedef float cnn_f32x4 __attribute__((ext_vector_type(4)));

template <int DT> struct CnnMcT;
template <> struct CnnMcT<kF32> {
    typedef float E;
    static constexpr int KS = 4;   // channels per step
    __device__ static float enc(float v) { return v; }
    __device__ static float dec(float e) { return e; }
};
template <> struct CnnMcT<kBF16> {
    typedef uint16_t E;
    static constexpr int KS = 16;
    __device__ static uint16_t enc(float v) { return (uint16_t)(__float_as_uint(cnn_round(v, kBF16)) >> 16); }
    __device__ static float dec(uint16_t e) { return __uint_as_float((uint32_t)e << 16); }
};
template <> struct CnnMcT<kF16> {
    typedef uint16_t E;
    static constexpr int KS = 16;
    __device__ static uint16_t enc(float v)
    {
        const _Float16 h = (_Float16)v;
        return *reinterpret_cast<const uint16_t *>(&h);
    }
    __device__ static float dec(uint16_t e) { return (float)*reinterpret_cast<const _Float16 *>(&e); }
};

__host__ __device__ inline size_t cnn_mc_lds_bytes(int B, int S, int F, int esz)
{
    const size_t rows = (size_t)B * S;
    size_t b = sizeof(float) * (rows + rows * F);        // x, h
    b = (b + 15) & ~(size_t)15;
    b += 2 * (size_t)esz * rows * F;                     // t, u
    b = (b + 15) & ~(size_t)15;
    b += sizeof(float) * (rows + 2 * (size_t)B) + 3 * sizeof(int) * (size_t)B;
    return b;
}

// one convolution of the batch: out = in (*) W + bias; GELU + store in the format, or add into h.  The 9 F
// products of an output are one contraction over the (offset, channel) index kk = k F + c: FP32 takes it 4 at a
// time (v_mfma_f32_16x16x4_f32, 4 channels of one offset), the 16-bit formats 32 at a time
// (v_mfma_f32_16x16x32_bf16 / _f16: lane group lk = lane / 16 holds kk = 32 step + 8 lk .. + 7, eight channels
// of one offset; for F = 16 the last step's second offset is past the ninth and reads zero).
template <int DT, int F, bool RESID>
__device__ inline void cnn_mc_conv(const typename CnnMcT<DT>::E *in, const void *wmc, const float *bias, int rows,
                                   int S, int L, typename CnnMcT<DT>::E *out, float *h)
{
    typedef CnnMcT<DT> M;
    typedef typename M::E E;
    static_assert(F == 16 || F == 32, "16 or 32 channels");
    constexpr int kSteps = (9 * F + 31) / 32;             // 32-deep steps of the 16-bit forms
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, la = lane & 15, lk = lane >> 4;
    const E *W = reinterpret_cast<const E *>(wmc);
    for (int mt = wave; mt < rows / 16; mt += kCnnThreads / 64) {
        const int row = mt * 16 + la, b = row / S, s = row - b * S;
        if constexpr (DT == kF32) {
            int nrow[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) nrow[k] = b * S + cnn_nbr(s, k, L);
#pragma unroll
            for (int nt = 0; nt < F / 16; ++nt) {
                cnn_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                const int o = nt * 16 + la;
#pragma unroll
                for (int k = 0; k < 9; ++k) {
#pragma unroll
                    for (int cs = 0; cs < F / M::KS; ++cs) {
                        const int c = cs * 4 + lk;
                        const float a = in[(size_t)nrow[k] * F + c];
                        const float w = W[((size_t)k * F + o) * F + c];
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w, acc, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int orow = mt * 16 + 4 * lk + r;
                    const float v = acc[r] + bias[o];
                    if constexpr (RESID) h[(size_t)orow * F + o] += v;
                    else out[(size_t)orow * F + o] = M::enc(cnn_round(cnn_gelu(v), DT));
                }
            }
        } else {
            // step st: F = 32, offset st, channels 8 lk .. 8 lk + 7; F = 16, offset 2 st + lk / 2, channels
            // 8 (lk % 2) .. + 7 (offset 9 of the last step is zero)
            int nrow[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) nrow[k] = b * S + cnn_nbr(s, k, L);
            const int c = F == 32 ? 8 * lk : 8 * (lk & 1), hi = lk >> 1;
#pragma unroll
            for (int nt = 0; nt < F / 16; ++nt) {
                cnn_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                const int o = nt * 16 + la;
#pragma unroll
                for (int st = 0; st < kSteps; ++st) {
                    int k, nr;
                    bool ok = true;
                    if constexpr (F == 32) {
                        k = st;
                        nr = nrow[st];
                    } else {
                        const int k0 = 2 * st, k1 = 2 * st + 1 < 9 ? 2 * st + 1 : 8;
                        k = hi ? k1 : k0;
                        nr = hi ? nrow[k1] : nrow[k0];
                        ok = 2 * st + 1 < 9 || !hi;
                    }
                    uint4 av = *reinterpret_cast<const uint4 *>(in + (size_t)nr * F + c);
                    const uint4 wv = *reinterpret_cast<const uint4 *>(W + ((size_t)k * F + o) * F + c);
                    if (!ok) av = make_uint4(0u, 0u, 0u, 0u);
                    if constexpr (DT == kBF16) {
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cnn_bf16x8, av),
                                                                      __builtin_bit_cast(cnn_bf16x8, wv), acc, 0, 0, 0);
                    } else {
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(cnn_h16x8, av),
                                                                     __builtin_bit_cast(cnn_h16x8, wv), acc, 0, 0, 0);
                    }
                }
                // D[i][j] of a 16 x 16 block: j = lane % 16, i = 4 (lane / 16) + register
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int orow = mt * 16 + 4 * lk + r;
                    const float v = acc[r] + bias[o];
                    if constexpr (RESID) h[(size_t)orow * F + o] += v;
                    else out[(size_t)orow * F + o] = M::enc(cnn_round(cnn_gelu(v), DT));
                }
            }
        }
    }
}

// log psi of the B configurations in x into f[B]; ends with a barrier
template <int DT, int F>
__device__ void cnn_mc_forward(const CnnDev &net, int B, float *x, float *h, typename CnnMcT<DT>::E *t,
                               typename CnnMcT<DT>::E *u, float *rsum, float *f)
{
    typedef CnnMcT<DT> M;
    const int L = net.L, S = L * L, rows = B * S, tid = threadIdx.x;
    const float *P = net.p;
    const int64_t per = 9 * (int64_t)F * F;
    const size_t esz = sizeof(typename M::E);
    for (int idx = tid; idx < rows * F; idx += kCnnThreads) {
        const int row = idx / F, o = idx - (idx / F) * F, b = row / S, s = row - b * S;
        float a = P[net.b0 + o];
        for (int k = 0; k < 9; ++k) a = fmaf(P[net.w0 + (int64_t)k * F + o], x[b * S + cnn_nbr(s, k, L)], a);
        h[idx] = a;
    }
    __syncthreads();
    for (int r = 0; r < net.R; ++r) {
        const float *g = P + net.g[r], *be = P + net.be[r];
        for (int row = tid; row < rows; row += kCnnThreads) {
            const float *hs = h + (size_t)row * F;
            float mu = 0.0f;
            for (int c = 0; c < F; ++c) mu += hs[c];
            mu /= (float)F;
            float var = 0.0f;
            for (int c = 0; c < F; ++c) var = fmaf(hs[c] - mu, hs[c] - mu, var);
            const float rs = 1.0f / sqrtf(var / (float)F + kLnEps);
            for (int c = 0; c < F; ++c)
                t[(size_t)row * F + c] = M::enc(cnn_round(cnn_gelu(fmaf((hs[c] - mu) * rs, g[c], be[c])), DT));
        }
        __syncthreads();
        cnn_mc_conv<DT, F, false>(t, (const char *)net.wmc + esz * (size_t)(2 * r) * per, P + net.b1[r], rows, S, L,
                                  u, h);
        __syncthreads();
        cnn_mc_conv<DT, F, true>(u, (const char *)net.wmc + esz * (size_t)(2 * r + 1) * per, P + net.b2[r], rows, S,
                                 L, u, h);
        __syncthreads();
    }
    const float *gf = P + net.gf, *bef = P + net.bef;
    for (int row = tid; row < rows; row += kCnnThreads) {
        const float *hs = h + (size_t)row * F;
        float mu = 0.0f;
        for (int c = 0; c < F; ++c) mu += hs[c];
        mu /= (float)F;
        float var = 0.0f;
        for (int c = 0; c < F; ++c) var = fmaf(hs[c] - mu, hs[c] - mu, var);
        const float rs = 1.0f / sqrtf(var / (float)F + kLnEps);
        float a = 0.0f;
        for (int c = 0; c < F; ++c) a += fmaf((hs[c] - mu) * rs, gf[c], bef[c]);
        rsum[row] = a;
    }
    __syncthreads();
    if (tid < B) {
        float a = 0.0f;
        for (int s = 0; s < S; ++s) a += rsum[tid * S + s];
        f[tid] = a;
    }
    __syncthreads();
}

template <int DT, int F>
__global__ void __launch_bounds__(kCnnThreads) cnn_sample_mc_kernel(CnnSampleArgs A, int B)
{
    typedef typename CnnMcT<DT>::E E;
    extern __shared__ __align__(16) unsigned char smc[];
    const int L = A.net.L, S = L * L, rows = B * S, tid = threadIdx.x;
    float *x = reinterpret_cast<float *>(smc);
    float *h = x + rows;
    size_t off = ((sizeof(float) * ((size_t)rows + (size_t)rows * F)) + 15) & ~(size_t)15;
    E *t = reinterpret_cast<E *>(smc + off);
    E *u = t + (size_t)rows * F;
    off = (off + 2 * sizeof(E) * (size_t)rows * F + 15) & ~(size_t)15;
    float *rsum = reinterpret_cast<float *>(smc + off);
    float *fcur = rsum + rows, *fnew = fcur + B;
    int *site = reinterpret_cast<int *>(fnew + B), *accn = site + B;
    uint32_t *ubs = reinterpret_cast<uint32_t *>(accn + B);
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * A.sweep_size;
    for (int64_t c0 = (int64_t)blockIdx.x * B; c0 < A.n_chains; c0 += (int64_t)gridDim.x * B) {
        for (int i = tid; i < rows; i += kCnnThreads) {
            const int64_t c = c0 + i / S;
            x[i] = c < A.n_chains ? (float)A.chain_state[c * S + i % S] : 1.0f;
        }
        if (tid < B) accn[tid] = 0;
        __syncthreads();
        cnn_mc_forward<DT, F>(A.net, B, x, h, t, u, rsum, fcur);
        for (int64_t k = 0; k < total; ++k) {
            const uint64_t step = A.step_offset + (uint64_t)k;
            if (tid < B) {
                const uint32_t gid = A.chain_id_offset + (uint32_t)(c0 + tid);
                const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, A.inst << 8, key0, key1);
                const int i = index_from_word(rb.r0, S);
                site[tid] = i;
                ubs[tid] = rb.r2 >> 8;
                x[tid * S + i] = -x[tid * S + i];
            }
            __syncthreads();
            cnn_mc_forward<DT, F>(A.net, B, x, h, t, u, rsum, fnew);
            if (tid < B) {
                const int64_t c = c0 + tid;
                const float d = 2.0f * (fnew[tid] - fcur[tid]);
                const float l2u = __builtin_amdgcn_logf((float)ubs[tid] * 5.9604644775390625e-8f);
                const bool accept = l2u < d * 1.4426950408889634f;
                if (accept) {
                    fcur[tid] = fnew[tid];
                    ++accn[tid];
                } else {
                    x[tid * S + site[tid]] = -x[tid * S + site[tid]];
                }
                if (c < A.n_traced) {
                    const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                    A.tr_site[idx] = site[tid] | (0xFFFF << 16);
                    A.tr_ubits[idx] = ubs[tid];
                    A.tr_delta[idx] = d;
                    A.tr_acc[idx] = accept ? 1 : 0;
                }
            }
            __syncthreads();
            if ((k + 1) % A.sweep_size == 0) {
                const int64_t out = (k + 1) / A.sweep_size - 1 - A.n_burnin;
                if (out >= 0) {
                    for (int i = tid; i < rows; i += kCnnThreads) {
                        const int64_t c = c0 + i / S;
                        if (c < A.n_chains && A.samples)
                            A.samples[((size_t)out * A.n_chains + c) * S + i % S] = x[i] > 0.0f ? 1 : -1;
                    }
                    if (A.logpsi && tid < B && c0 + tid < A.n_chains)
                        A.logpsi[(size_t)out * A.n_chains + c0 + tid] = fcur[tid];
                    __syncthreads();
                }
            }
        }
        for (int i = tid; i < rows; i += kCnnThreads) {
            const int64_t c = c0 + i / S;
            if (c < A.n_chains) A.chain_state[c * S + i % S] = x[i] > 0.0f ? 1 : -1;
        }
        if (A.n_acc && tid < B && c0 + tid < A.n_chains) A.n_acc[c0 + tid] = (unsigned long long)accn[tid];
        __syncthreads();
    }
}

// Chains per workgroup for the matrix-core sampler (0: not applicable): B * S a
// multiple of 16 and the batch's activations within 160 KB of LDS.
static int cnn_mc_chains(const CnnDev &net)
{
    if (net.F != 16 && net.F != 32) return 0;
    const int S = net.L * net.L;
    const int esz = net.dtype == NQS_F32 ? 4 : 2;
    for (int B : {16, 8, 4, 2, 1})
        if ((B * S) % 16 == 0 && cnn_mc_lds_bytes(B, S, net.F, esz) <= 160 * 1024) return B;
    return 0;
}

template <int DT>
static void launch_cnn_mc(const CnnSampleArgs &A, int B, int64_t blocks, size_t lds, hipStream_t stream)
{
    if (A.net.F == 16) {
        allow_lds(cnn_sample_mc_kernel<DT, 16>, lds);
        hipLaunchKernelGGL((cnn_sample_mc_kernel<DT, 16>), dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, A, B);
    } else {
        allow_lds(cnn_sample_mc_kernel<DT, 32>, lds);
        hipLaunchKernelGGL((cnn_sample_mc_kernel<DT, 32>), dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, A, B);
    }
}

// ---- host ----

static nqs_status cnn_check(const CnnDev &net)
{
    if (cnn_lds_bytes(net.L * net.L, net.F) > 160 * 1024)
        return set_error(NQS_EUNSUPPORTED, "convolutional network activations exceed 160 KB of LDS (L^2 x F too large)");
    return NQS_OK;
}

nqs_status cnn_logpsi(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const CnnDev &net = m->copies[NQS_F32].cnn;
    if ((st = cnn_check(net)) != NQS_OK) return st;
    const size_t lds = cnn_lds_bytes(net.L * net.L, net.F);
    allow_lds(cnn_logpsi_kernel, lds);
    const int64_t blocks = std::min<int64_t>(n, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(cnn_logpsi_kernel, dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, net, samples, n, logpsi);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status cnn_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                      uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, cfg.dtype, stream);
    if (st != NQS_OK) return st;
    const CnnDev &net = m->copies[cfg.dtype].cnn;
    if ((st = cnn_check(net)) != NQS_OK) return st;
    const int S = net.L * net.L;
    if (cfg.init_chains) {
        st = launch_init_chains(chain_state, cfg.n_chains, S, NQS_MOVE_FLIP, cfg.seed, cfg.instance_id,
                                cfg.chain_id_offset, stream);
        if (st != NQS_OK) return st;
    }
    CnnSampleArgs A;
    A.net = net;
    A.chain_state = chain_state;
    A.samples = samples;
    A.logpsi = logpsi;
    A.n_acc = (unsigned long long *)n_accepted;
    A.n_chains = cfg.n_chains;
    A.n_sweeps = cfg.n_sweeps;
    A.n_burnin = cfg.n_burnin;
    A.sweep_size = cfg.sweep_size > 0 ? cfg.sweep_size : S;
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
    const int B = cfg.lanes_per_chain == -1 ? 0 : cnn_mc_chains(net);
    if (B > 0) {
        const size_t lds = cnn_mc_lds_bytes(B, S, net.F, net.dtype == NQS_F32 ? 4 : 2);
        const int64_t groups = (cfg.n_chains + B - 1) / B;
        const int64_t blocks = std::min<int64_t>(groups, (int64_t)device_cus() * 16);
        if (net.dtype == NQS_BF16) launch_cnn_mc<kBF16>(A, B, blocks, lds, stream);
        else if (net.dtype == NQS_F16) launch_cnn_mc<kF16>(A, B, blocks, lds, stream);
        else launch_cnn_mc<kF32>(A, B, blocks, lds, stream);
        NQS_HIP_TRY(hipGetLastError());
        return NQS_OK;
    }
    const size_t lds = cnn_lds_bytes(S, net.F);
    allow_lds(cnn_sample_kernel, lds);
    const int64_t blocks = std::min<int64_t>(cfg.n_chains, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(cnn_sample_kernel, dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, A);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status cnn_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                            double *eloc, hipStream_t stream)
{
    if (ham.kind != NQS_TFIM || ham.dim != 2 || ham.L != m->desc.lat_L || !ham.pbc)
        return set_error(NQS_EUNSUPPORTED,
                         "convolutional-network local energies: TFIM on the network's periodic L x L lattice");
    nqs_status st = ensure_copy(m, dtype, stream);
    if (st != NQS_OK) return st;
    const CnnDev &net = m->copies[dtype].cnn;
    if ((st = cnn_check(net)) != NQS_OK) return st;
    const size_t lds = cnn_lds_bytes(net.L * net.L, net.F);
    allow_lds(cnn_eloc_tfim_kernel, lds);
    const int64_t blocks = std::min<int64_t>(n, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(cnn_eloc_tfim_kernel, dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, net, samples, n,
                       ham.J, ham.h, eloc);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---- log-derivatives O = d log psi / d theta (Eq. eq:forces), FP32 copy ----
//
// One sample per workgroup.  The forward pass keeps the residual stream before
// every block and after the last, each block's conv1 pre-activation and the
// layer-norm statistics in LDS; the backward pass recomputes phi(LN h) and
// phi(conv1) from them.  Every derivative is a fixed-order sum over sites.

__device__ inline float cnn_gelu_grad(float z)
{
    const float c = 0.7978845608028654f;
    const float a = c * fmaf(0.044715f * z * z, z, z);
    const float th = tanhf(a);
    return 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * c * fmaf(3.0f * 0.044715f, z * z, 1.0f);
}

__host__ __device__ inline size_t cnn_grad_lds_bytes(int S, int F, int R)
{
    const size_t SF = (size_t)S * F;
    return sizeof(float) * ((size_t)S + (size_t)(2 * R + 1) * SF + 2 * (size_t)(R + 1) * S + 4 * SF +
                            kCnnThreads / 64);
}

// per-site layer-norm statistics of h into mu[s], rs[s]
__device__ inline void cnn_ln_stats(const float *h, int S, int F, float *mu, float *rs)
{
    for (int s = threadIdx.x; s < S; s += kCnnThreads) {
        const float *hs = h + (size_t)s * F;
        float m = 0.0f;
        for (int c = 0; c < F; ++c) m += hs[c];
        m /= (float)F;
        float v = 0.0f;
        for (int c = 0; c < F; ++c) v = fmaf(hs[c] - m, hs[c] - m, v);
        mu[s] = m;
        rs[s] = 1.0f / sqrtf(v / (float)F + kLnEps);
    }
}

// gh[s][:] += LN backward of gz (gradient at the layer-norm output) through scale g
__device__ inline void cnn_ln_back(const float *h, const float *mu, const float *rs, const float *gz, const float *g,
                                   int S, int F, float *gh)
{
    for (int s = threadIdx.x; s < S; s += kCnnThreads) {
        const float *hs = h + (size_t)s * F, *gs = gz + (size_t)s * F;
        float m1 = 0.0f, m2 = 0.0f;
        for (int c = 0; c < F; ++c) {
            const float gn = gs[c] * g[c];
            m1 += gn;
            m2 = fmaf(gn, (hs[c] - mu[s]) * rs[s], m2);
        }
        m1 /= (float)F;
        m2 /= (float)F;
        for (int c = 0; c < F; ++c) {
            const float gn = gs[c] * g[c], nh = (hs[c] - mu[s]) * rs[s];
            gh[(size_t)s * F + c] += rs[s] * (gn - m1 - nh * m2);
        }
    }
}

// O[off + (o*C + c)*9 + k] = sum_s g[s][o] in[nbr(s,k)][c];  O[boff + o] = sum_s g[s][o]
__device__ inline void cnn_wgrad(const float *g, const float *in, int S, int L, int C, int F, float *O, int64_t off,
                                 int64_t boff)
{
    const int n = 9 * C * F;
    for (int q = threadIdx.x; q < n + F; q += kCnnThreads) {
        if (q < n) {
            const int o = q / (9 * C), r = q - o * 9 * C, c = r / 9, k = r - c * 9;
            float a = 0.0f;
            for (int s = 0; s < S; ++s) a = fmaf(g[(size_t)s * F + o], in[(size_t)cnn_nbr(s, k, L) * C + c], a);
            O[off + q] = a;
        } else {
            const int o = q - n;
            float a = 0.0f;
            for (int s = 0; s < S; ++s) a += g[(size_t)s * F + o];
            O[boff + o] = a;
        }
    }
}

// gin[s'][c] = sum_{k,o} W[c][k][o] g[nbr(s', 8 - k)][o]   (the transposed convolution)
__device__ inline void cnn_inback(const float *__restrict__ W, const float *g, int S, int L, int F, float *gin)
{
    for (int idx = threadIdx.x; idx < S * F; idx += kCnnThreads) {
        const int s = idx / F, c = idx - (idx / F) * F;
        float a = 0.0f;
        for (int k = 0; k < 9; ++k) {
            const float *gs = g + (size_t)cnn_nbr(s, 8 - k, L) * F;
            const float *w = W + ((size_t)c * 9 + k) * F;
            for (int o = 0; o < F; ++o) a = fmaf(w[o], gs[o], a);
        }
        gin[idx] = a;
    }
}

__global__ void __launch_bounds__(kCnnThreads) cnn_grad_kernel(CnnDev net, const int8_t *__restrict__ samples,
                                                               int64_t n, int64_t P, float *__restrict__ logpsi,
                                                               float *__restrict__ O)
{
    extern __shared__ float sm[];
    const int L = net.L, S = L * L, F = net.F, R = net.R, tid = threadIdx.x;
    const size_t SF = (size_t)S * F;
    float *x = sm;
    float *H = x + S;                       // [R+1][S][F]
    float *A1 = H + (size_t)(R + 1) * SF;   // [R][S][F]
    float *MU = A1 + (size_t)R * SF;        // [R+1][S]
    float *RS = MU + (size_t)(R + 1) * S;   // [R+1][S]
    float *gh = RS + (size_t)(R + 1) * S;   // [S][F]
    float *gu = gh + SF;
    float *T1 = gu + SF;
    float *T2 = T1 + SF;
    float *red = T2 + SF;
    const float *Pp = net.p;
    for (int64_t row = blockIdx.x; row < n; row += gridDim.x) {
        float *Orow = O ? O + row * P : nullptr;
        for (int i = tid; i < S; i += kCnnThreads) x[i] = (float)samples[row * S + i];
        __syncthreads();
        // forward, keeping what the backward pass needs
        for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
            const int s = idx / F, o = idx - (idx / F) * F;
            H[idx] = cnn_conv_at(Pp + net.w0, Pp + net.b0, x, s, o, L, 1, F);
        }
        __syncthreads();
        for (int r = 0; r < R; ++r) {
            const float *h = H + (size_t)r * SF;
            cnn_ln_stats(h, S, F, MU + (size_t)r * S, RS + (size_t)r * S);
            __syncthreads();
            const float *g = Pp + net.g[r], *be = Pp + net.be[r];
            for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
                const int s = idx / F, c = idx - (idx / F) * F;
                T1[idx] = cnn_gelu(fmaf((h[idx] - MU[r * S + s]) * RS[r * S + s], g[c], be[c]));
            }
            __syncthreads();
            float *a1 = A1 + (size_t)r * SF;
            for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
                const int s = idx / F, o = idx - (idx / F) * F;
                const float a = cnn_conv_at(Pp + net.w1[r], Pp + net.b1[r], T1, s, o, L, F, F);
                a1[idx] = a;
                T2[idx] = cnn_gelu(a);
            }
            __syncthreads();
            float *hn = H + (size_t)(r + 1) * SF;
            for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
                const int s = idx / F, o = idx - (idx / F) * F;
                hn[idx] = h[idx] + cnn_conv_at(Pp + net.w2[r], Pp + net.b2[r], T2, s, o, L, F, F);
            }
            __syncthreads();
        }
        const float *hR = H + (size_t)R * SF;
        float *muR = MU + (size_t)R * S, *rsR = RS + (size_t)R * S;
        cnn_ln_stats(hR, S, F, muR, rsR);
        __syncthreads();
        const float *gf = Pp + net.gf, *bef = Pp + net.bef;
        float part = 0.0f;
        for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
            const int s = idx / F, c = idx - (idx / F) * F;
            part += fmaf((hR[idx] - muR[s]) * rsR[s], gf[c], bef[c]);
        }
        part = group_sum<64>(part);
        if ((tid & 63) == 0) red[tid >> 6] = part;
        __syncthreads();
        if (tid == 0 && logpsi) {
            float f = 0.0f;
            for (int w = 0; w < kCnnThreads / 64; ++w) f += red[w];
            logpsi[row] = f;
        }
        if (Orow) {
            // readout: d/d gamma_f, d/d beta_f; gradient at the final layer-norm output is 1
            for (int c = tid; c < F; c += kCnnThreads) {
                float a = 0.0f;
                for (int s = 0; s < S; ++s) a += (hR[(size_t)s * F + c] - muR[s]) * rsR[s];
                Orow[net.gf + c] = a;
                Orow[net.bef + c] = (float)S;
            }
            for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
                gu[idx] = 1.0f;
                gh[idx] = 0.0f;
            }
            __syncthreads();
            cnn_ln_back(hR, muR, rsR, gu, gf, S, F, gh);
            __syncthreads();
            for (int r = R - 1; r >= 0; --r) {
                const float *h = H + (size_t)r * SF, *a1 = A1 + (size_t)r * SF;
                const float *mu = MU + (size_t)r * S, *rs = RS + (size_t)r * S;
                const float *g = Pp + net.g[r], *be = Pp + net.be[r];
                for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
                    const int s = idx / F, c = idx - (idx / F) * F;
                    T1[idx] = cnn_gelu(fmaf((h[idx] - mu[s]) * rs[s], g[c], be[c]));   // t
                    T2[idx] = cnn_gelu(a1[idx]);                                        // u
                }
                __syncthreads();
                // conv2: weights from gh and u; gradient at u
                cnn_wgrad(gh, T2, S, L, F, F, Orow, net.w2[r], net.b2[r]);
                cnn_inback(Pp + net.w2[r], gh, S, L, F, gu);
                __syncthreads();
                for (int idx = tid; idx < (int)SF; idx += kCnnThreads) gu[idx] *= cnn_gelu_grad(a1[idx]);
                __syncthreads();
                // conv1: weights from the conv1 gradient and t; gradient at t (into T2)
                cnn_wgrad(gu, T1, S, L, F, F, Orow, net.w1[r], net.b1[r]);
                cnn_inback(Pp + net.w1[r], gu, S, L, F, T2);
                __syncthreads();
                // through phi and the block's layer norm (scale and shift), into gh
                for (int idx = tid; idx < (int)SF; idx += kCnnThreads) {
                    const int s = idx / F, c = idx - (idx / F) * F;
                    T2[idx] *= cnn_gelu_grad(fmaf((h[idx] - mu[s]) * rs[s], g[c], be[c]));
                }
                __syncthreads();
                for (int c = tid; c < F; c += kCnnThreads) {
                    float ag = 0.0f, ab = 0.0f;
                    for (int s = 0; s < S; ++s) {
                        const float gz = T2[(size_t)s * F + c];
                        ag = fmaf(gz, (h[(size_t)s * F + c] - mu[s]) * rs[s], ag);
                        ab += gz;
                    }
                    Orow[net.g[r] + c] = ag;
                    Orow[net.be[r] + c] = ab;
                }
                cnn_ln_back(h, mu, rs, T2, g, S, F, gh);
                __syncthreads();
            }
            cnn_wgrad(gh, x, S, L, 1, F, Orow, net.w0, net.b0);
        }
        __syncthreads();
    }
}

nqs_status cnn_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                           const float *vjp_in, float *vjp_out, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const CnnDev &net = m->copies[NQS_F32].cnn;
    const int S = net.L * net.L;
    const size_t lds = cnn_grad_lds_bytes(S, net.F, net.R);
    if (lds > 160 * 1024)
        return set_error(NQS_EUNSUPPORTED, "convolutional-network gradient: activations exceed 160 KB of LDS");
    allow_lds(cnn_grad_kernel, lds);
    const int64_t P = m->P;
    if (logpsi || O) {
        const int64_t blocks = std::min<int64_t>(n, (int64_t)device_cus() * 16);
        hipLaunchKernelGGL(cnn_grad_kernel, dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, net, samples, n, P,
                           logpsi, O);
        NQS_HIP_TRY(hipGetLastError());
    }
    if (vjp_in) {
        // vjp_out = O^T vjp_in through blocks of rows of O in the workspace
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(256ll << 20) / (P * 4)));
        float *Ow = (float *)workspace(sizeof(float) * (size_t)chunk * P, stream);
        if (!Ow) return set_error(NQS_ENOMEM, "workspace allocation failed");
        for (int64_t k0 = 0; k0 < n; k0 += chunk) {
            const int64_t kn = std::min(chunk, n - k0);
            const int64_t blocks = std::min<int64_t>(kn, (int64_t)device_cus() * 16);
            hipLaunchKernelGGL(cnn_grad_kernel, dim3((unsigned)blocks), dim3(kCnnThreads), lds, stream, net,
                               samples + k0 * S, kn, P, nullptr, Ow);
            st = launch_vjp_chunk(Ow, vjp_in + k0, kn, P, vjp_out, k0 == 0, stream);
            if (st != NQS_OK) return st;
        }
    }
    return NQS_OK;
}

}  // namespace nqs
