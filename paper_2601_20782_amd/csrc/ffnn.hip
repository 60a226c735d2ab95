// Dense networks: h_l = ReLU(W_l h_{l-1} + b_l) for l < L, log psi = sum log cosh(z_L).
// This file builds the reduced-precision copies and holds the log-derivative
// (backward) kernel; the MFMA sampler and local energies live in ffnn_mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "ffnn_reg.h"
#include "internal.h"

namespace nqs {

// ---------------------------------------------------------------------------
// Copy builder.  For every layer: the format-rounded weights as FP32 values
// in both orientations and FP32 biases.  For the matrix-core path the second
// layer is also kept zero-padded to [ceil(w2/64)*64][ceil(w1/16)*16] (FP32
// values and raw 16-bit codes), and the first layer transposed, [N][w1 pad],
// as raw codes for the LDS-resident rank-1/2 updates.
// ---------------------------------------------------------------------------
__global__ void ffnn_round_layer_kernel(const double *__restrict__ Wsrc, const double *__restrict__ bsrc, int out,
                                        int in, int dtype, float *W, float *Wt, float *b)
{
    const int64_t n = (int64_t)out * in;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n + out; p += (int64_t)gridDim.x * blockDim.x) {
        if (p < n) {
            const int r = (int)(p / in), k = (int)(p % in);
            const float v = (float)round_to_dtype(Wsrc[p], dtype);
            W[p] = v;
            Wt[(int64_t)k * out + r] = v;
        } else {
            b[p - n] = (float)round_to_dtype(bsrc[p - n], dtype);
        }
    }
}

// dst[r][c] (ld_dst, zero padded to rows_p x cols_p) from src[r][c] (ld_src)
__global__ void ffnn_pad_kernel(const float *__restrict__ src, int rows, int cols, int ld_src, int rows_p, int cols_p,
                                int dtype, uint16_t *codes, float *f32)
{
    const int64_t n = (int64_t)rows_p * cols_p;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(p / cols_p), c = (int)(p % cols_p);
        const float v = (r < rows && c < cols) ? src[(int64_t)r * ld_src + c] : 0.0f;
        if (f32) f32[p] = v;
        if (codes) {
            uint16_t code;
            if (dtype == kF16) {
                const _Float16 h = (_Float16)v;   // exact: v is an f16 value
                memcpy(&code, &h, 2);
            } else {
                code = (uint16_t)(__float_as_uint(v) >> 16);   // exact: v is a bf16 value
            }
            codes[p] = code;
        }
    }
}

// ---------------------------------------------------------------------------
// FP8 (E4M3) copy.  Every weight tensor W_l and bias b_l has its own scale
// amax/448 (FP32) and values q * scale, q an E4M3 code (the downcast of the
// two-copy scheme, App. A extended to FP8).  The matrix cores multiply the
// codes: W_l as [Np][Kp] bytes, the layer input as codes of the spins (+-1,
// exact) or of h_{l-1} / s_l, where s_l = 2^ceil(log2(B_l / 448)) and B_l
// bounds |h_l| over every configuration (B_0 = 1, B_l = max_k sum_i
// |W_l[k,i]| B_{l-1} + |b_l[k]| on the rounded values), so no scaled input
// exceeds 448.  The products are accumulated in FP32 and scaled back by
// sW_l s_l.
// ---------------------------------------------------------------------------

// OCP E4M3 code of a value that is exactly representable in the format.
__device__ __forceinline__ uint8_t e4m3_code_exact(double q)
{
    const uint32_t sign = q < 0.0 || (q == 0.0 && signbit(q)) ? 0x80u : 0u;
    const double a = fabs(q);
    if (a == 0.0) return (uint8_t)sign;
    int e;
    const double m = frexp(a, &e);            // a = m 2^e, m in [0.5, 1)
    const int E = e - 1;                      // a = (2m) 2^E, 2m in [1, 2)
    if (E < -6) return (uint8_t)(sign | (uint32_t)(a * 512.0));        // subnormal: a / 2^-9
    return (uint8_t)(sign | ((uint32_t)(E + 7) << 3) | (uint32_t)((2.0 * m - 1.0) * 8.0));
}

// codes[Np][Kp] of W[out][in] / scale (zero padded) and the transposed FP32 values
__global__ void ffnn_e4m3_codes_kernel(const double *__restrict__ W, int out, int in,
                                       const unsigned long long *__restrict__ amax_bits, int Np, int Kp,
                                       uint8_t *__restrict__ codes, float *__restrict__ Wt)
{
    const double amax = __longlong_as_double((long long)*amax_bits);
    const float scale = amax > 0.0 ? (float)(amax / 448.0) : 1.0f;
    const int64_t n = (int64_t)Np * Kp;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(p / Kp), c = (int)(p % Kp);
        uint8_t code = 0;
        if (r < out && c < in) {
            const double q = round_to_dtype(W[(int64_t)r * in + c] / (double)scale, kE4M3);
            code = e4m3_code_exact(q);
            Wt[(int64_t)c * out + r] = (float)(q * (double)scale);
        }
        codes[p] = code;
    }
}

// Per row k of W (one wave each): rs[k] = sum_i |q_ki| and bq[k] = |q_bk|, with q the E4M3 values
// before scaling (multiples of 2^-9 below 448: the FP64 sums are exact in any order).
__global__ void ffnn_e4m3_rowsum_kernel(const double *__restrict__ W, const double *__restrict__ b, int out, int in,
                                        const unsigned long long *__restrict__ amax_w,
                                        const unsigned long long *__restrict__ amax_b, double *rs, double *bq)
{
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= out) return;
    const double aw = __longlong_as_double((long long)*amax_w), ab = __longlong_as_double((long long)*amax_b);
    const float sw = aw > 0.0 ? (float)(aw / 448.0) : 1.0f, sb = ab > 0.0 ? (float)(ab / 448.0) : 1.0f;
    double acc = 0.0;
    for (int c = lane; c < in; c += 64) acc += fabs(round_to_dtype(W[(int64_t)r * in + c] / (double)sw, kE4M3));
    acc = group_sum<64>(acc);
    if (lane == 0) {
        rs[r] = acc;
        bq[r] = fabs(round_to_dtype(b[r] / (double)sb, kE4M3));
    }
}

static nqs_status ffnn_build_e4m3(nqs_model *m, hipStream_t stream)
{
    const nqs_model_desc &d = m->desc;
    Copy &c = m->copies[NQS_FP8_E4M3];
    FfnnDev &f = c.ffnn;
    const int L = d.n_layers;
    f.n_layers = L;
    f.widths[0] = d.n_visible;
    for (int l = 0; l < L; ++l) f.widths[l + 1] = d.widths[l];
    f.m1p = f.m2p = 0;   // the two-layer register kernels take 16-bit copies only
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t bytes = al(sizeof(unsigned long long) * 2 * L);
    for (int l = 0; l < L; ++l) {
        const size_t n = (size_t)f.widths[l + 1] * f.widths[l];
        f.Kp[l] = (f.widths[l] + 127) / 128 * 128;   // 128 one-byte codes per contraction step
        f.Np[l] = (f.widths[l + 1] + 127) / 128 * 128;
        bytes += 2 * al(sizeof(float) * n) + al(sizeof(float) * f.widths[l + 1]) + al((size_t)f.Np[l] * f.Kp[l]) +
                 al(sizeof(float) * f.Np[l]) + 2 * al(sizeof(double) * f.widths[l + 1]);
    }
    if (!c.block) NQS_HIP_TRY(hipMalloc(&c.block, bytes));
    char *base = (char *)c.block;
    auto carve = [&](size_t sz) {
        char *p = base;
        base += al(sz);
        return p;
    };
    unsigned long long *amax = (unsigned long long *)carve(sizeof(unsigned long long) * 2 * L);
    double *rs[NQS_MAX_LAYERS], *bq[NQS_MAX_LAYERS];
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        const int out = f.widths[l + 1], in = f.widths[l];
        const int64_t n = (int64_t)out * in;
        f.W[l] = (float *)carve(sizeof(float) * n);
        f.Wt[l] = (float *)carve(sizeof(float) * n);
        f.b[l] = (float *)carve(sizeof(float) * out);
        f.Wd[l] = carve((size_t)f.Np[l] * f.Kp[l]);
        f.bd[l] = (float *)carve(sizeof(float) * f.Np[l]);
        rs[l] = (double *)carve(sizeof(double) * out);
        bq[l] = (double *)carve(sizeof(double) * out);
        const double *Wm = m->master + off, *bm = m->master + off + n;
        nqs_status e = launch_e4m3_tensor(Wm, n, amax + 2 * l, f.W[l], stream);
        if (e != NQS_OK) return e;
        e = launch_e4m3_tensor(bm, out, amax + 2 * l + 1, f.b[l], stream);
        if (e != NQS_OK) return e;
        const int64_t nc = (int64_t)f.Np[l] * f.Kp[l];
        hipLaunchKernelGGL(ffnn_e4m3_codes_kernel, dim3((unsigned)std::min<int64_t>((nc + 255) / 256, 8192)), dim3(256),
                           0, stream, Wm, out, in, (const unsigned long long *)(amax + 2 * l), f.Np[l], f.Kp[l],
                           (uint8_t *)f.Wd[l], f.Wt[l]);
        hipLaunchKernelGGL(ffnn_pad_kernel, dim3((f.Np[l] + 255) / 256), dim3(256), 0, stream, f.b[l], 1, out, out, 1,
                           f.Np[l], (int)kF32, (uint16_t *)nullptr, f.bd[l]);
        hipLaunchKernelGGL(ffnn_e4m3_rowsum_kernel, dim3((out + 3) / 4), dim3(256), 0, stream, Wm, bm, out, in,
                           (const unsigned long long *)(amax + 2 * l), (const unsigned long long *)(amax + 2 * l + 1),
                           rs[l], bq[l]);
        NQS_HIP_TRY(hipGetLastError());
        off += n + out;
    }
    if ((size_t)(base - (char *)c.block) > bytes) return set_error(NQS_EDEVICE, "internal layout overflow");
    // scales on the host: weight scales from the amax words, input scales from the bounds B_l
    std::vector<unsigned long long> hmax(2 * L);
    NQS_HIP_TRY(hipMemcpyAsync(hmax.data(), amax, sizeof(unsigned long long) * 2 * L, hipMemcpyDeviceToHost, stream));
    std::vector<std::vector<double>> hrs(L), hbq(L);
    for (int l = 0; l + 1 < L; ++l) {
        hrs[l].resize(f.widths[l + 1]);
        hbq[l].resize(f.widths[l + 1]);
        NQS_HIP_TRY(hipMemcpyAsync(hrs[l].data(), rs[l], sizeof(double) * f.widths[l + 1], hipMemcpyDeviceToHost, stream));
        NQS_HIP_TRY(hipMemcpyAsync(hbq[l].data(), bq[l], sizeof(double) * f.widths[l + 1], hipMemcpyDeviceToHost, stream));
    }
    NQS_HIP_TRY(hipStreamSynchronize(stream));
    auto scale_of = [](unsigned long long bits) {
        double a;
        std::memcpy(&a, &bits, sizeof(double));
        return a > 0.0 ? (float)(a / 448.0) : 1.0f;
    };
    double B = 1.0;          // bound on |input of layer l| (spins)
    float s_in = 1.0f;       // scale of the input of layer l
    for (int l = 0; l < L; ++l) {
        const float sw = scale_of(hmax[2 * l]), sb = scale_of(hmax[2 * l + 1]);
        f.acc_scale[l] = sw * s_in;   // s_in is a power of two: exact
        if (l + 1 < L) {
            double Bn = 0.0;
            for (int k = 0; k < f.widths[l + 1]; ++k)
                Bn = std::max(Bn, ((double)sw * hrs[l][k]) * B + (double)sb * hbq[l][k]);
            const float s_next = Bn > 0.0 ? (float)std::ldexp(1.0, (int)std::ceil(std::log2(Bn / 448.0))) : 1.0f;
            f.next_inv[l] = 1.0f / s_next;   // exact: a power of two
            B = Bn;
            s_in = s_next;
        } else {
            f.next_inv[l] = 1.0f;
        }
    }
    c.valid = true;
    return NQS_OK;
}

nqs_status ffnn_build_copy(nqs_model *m, int dtype, hipStream_t stream)
{
    const nqs_model_desc &d = m->desc;
    if (dtype == NQS_FP8_E4M3) return ffnn_build_e4m3(m, stream);
    Copy &c = m->copies[dtype];
    FfnnDev &f = c.ffnn;
    f.n_layers = d.n_layers;
    f.widths[0] = d.n_visible;
    for (int l = 0; l < d.n_layers; ++l) f.widths[l + 1] = d.widths[l];
    const bool lp = dtype == NQS_BF16 || dtype == NQS_F16;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int N = f.widths[0], M1 = f.widths[1];
    f.m1p = (M1 + 63) / 64 * 64;   // lane k of a wave owns hidden units k + 64 q
    f.m2p = f.n_layers >= 2 ? (f.widths[2] + 63) / 64 * 64 : 0;
    size_t bytes = 0;
    for (int l = 0; l < f.n_layers; ++l) {
        const size_t n = (size_t)f.widths[l + 1] * f.widths[l];
        bytes += 2 * al(sizeof(float) * n) + al(sizeof(float) * f.widths[l + 1]);
    }
    if (f.n_layers >= 2)
        bytes += al(sizeof(uint16_t) * (size_t)f.m2p * f.m1p) + al(sizeof(uint16_t) * (size_t)N * f.m1p) +
                 al(sizeof(float) * (size_t)f.m2p * f.m1p) + al(sizeof(float) * (size_t)N * f.m1p) +
                 al(sizeof(float) * f.m1p) + al(sizeof(float) * f.m2p);
    const size_t esize = lp ? sizeof(uint16_t) : sizeof(float);
    for (int l = 0; l < f.n_layers; ++l) {
        f.Kp[l] = (f.widths[l] + 63) / 64 * 64;
        f.Np[l] = (f.widths[l + 1] + 127) / 128 * 128;
        bytes += al(esize * (size_t)f.Np[l] * f.Kp[l]) + al(sizeof(float) * f.Np[l]);
    }
    if (!c.block) NQS_HIP_TRY(hipMalloc(&c.block, bytes));
    char *base = (char *)c.block;
    auto carve = [&](size_t sz) {
        char *p = base;
        base += al(sz);
        return p;
    };
    for (int l = 0; l < f.n_layers; ++l) {
        const size_t n = (size_t)f.widths[l + 1] * f.widths[l];
        f.W[l] = (float *)carve(sizeof(float) * n);
        f.Wt[l] = (float *)carve(sizeof(float) * n);
        f.b[l] = (float *)carve(sizeof(float) * f.widths[l + 1]);
    }
    int64_t off = 0;
    for (int l = 0; l < f.n_layers; ++l) {
        const int out = f.widths[l + 1], in = f.widths[l];
        const int64_t n = (int64_t)out * in;
        const int blocks = (int)std::min<int64_t>((n + out + 255) / 256, 8192);
        hipLaunchKernelGGL(ffnn_round_layer_kernel, dim3(blocks), dim3(256), 0, stream, m->master + off,
                           m->master + off + n, out, in, dtype, f.W[l], f.Wt[l], f.b[l]);
        NQS_HIP_TRY(hipGetLastError());
        off += n + out;
    }
    if (f.n_layers >= 2) {
        const int M2 = f.widths[2];
        f.W2c = (uint16_t *)carve(sizeof(uint16_t) * (size_t)f.m2p * f.m1p);
        f.W1ct = (uint16_t *)carve(sizeof(uint16_t) * (size_t)N * f.m1p);
        f.W2p = (float *)carve(sizeof(float) * (size_t)f.m2p * f.m1p);
        f.W1tp = (float *)carve(sizeof(float) * (size_t)N * f.m1p);
        f.b1p = (float *)carve(sizeof(float) * f.m1p);
        f.b2p = (float *)carve(sizeof(float) * f.m2p);
        auto pad = [&](const float *src, int rows, int cols, int ld, int rows_p, int cols_p, uint16_t *codes,
                       float *f32) {
            const int64_t n = (int64_t)rows_p * cols_p;
            const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
            hipLaunchKernelGGL(ffnn_pad_kernel, dim3(blocks), dim3(256), 0, stream, src, rows, cols, ld, rows_p, cols_p,
                               dtype, codes, f32);
        };
        pad(f.W[1], M2, M1, M1, f.m2p, f.m1p, lp ? f.W2c : nullptr, f.W2p);
        pad(f.Wt[0], N, M1, M1, N, f.m1p, lp ? f.W1ct : nullptr, f.W1tp);
        pad(f.b[0], 1, M1, M1, 1, f.m1p, nullptr, f.b1p);
        pad(f.b[1], 1, M2, M2, 1, f.m2p, nullptr, f.b2p);
        NQS_HIP_TRY(hipGetLastError());
    }
    for (int l = 0; l < f.n_layers; ++l) {
        const int out = f.widths[l + 1], in = f.widths[l];
        f.Wd[l] = carve(esize * (size_t)f.Np[l] * f.Kp[l]);
        f.bd[l] = (float *)carve(sizeof(float) * f.Np[l]);
        const int64_t n = (int64_t)f.Np[l] * f.Kp[l];
        const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL(ffnn_pad_kernel, dim3(blocks), dim3(256), 0, stream, f.W[l], out, in, in, f.Np[l], f.Kp[l],
                           dtype, lp ? (uint16_t *)f.Wd[l] : nullptr, lp ? nullptr : (float *)f.Wd[l]);
        hipLaunchKernelGGL(ffnn_pad_kernel, dim3((f.Np[l] + 255) / 256), dim3(256), 0, stream, f.b[l], 1, out, out, 1,
                           f.Np[l], dtype, (uint16_t *)nullptr, f.bd[l]);
        NQS_HIP_TRY(hipGetLastError());
    }
    NQS_HIP_TRY(hipStreamSynchronize(stream));
    c.valid = true;
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// log psi and O_k by reverse-mode differentiation written out by hand.
// One block per sample (grid-stride); activations stay in LDS.
//   delta_L = tanh(z_L);  O_{b_l} = delta_l;  O_{W_l} = delta_l (x) h_{l-1};
//   delta_{l-1} = (W_l^T delta_l) * [z_{l-1} > 0]   (ReLU'(0) = 0).
// O rows are written with consecutive threads on consecutive parameters.
// ---------------------------------------------------------------------------
struct GradArgs {
    FfnnDev net;
    const int8_t *samples;
    int64_t n;
    float *logpsi;
    float *O;         // columns [p0, p1) of O, row stride p1 - p0
    int64_t P;
    int64_t p0, p1;
    float *acts;      // factor kernel: [n][sum of layer inputs] inputs a_{l-1} of every layer, post-ReLU
    float *dels;      // factor kernel: [n][sum of layer outputs] backpropagated deltas
    int lds_stride;   // floats reserved per layer activation vector
};

__global__ void __launch_bounds__(256) ffnn_grad_kernel(GradArgs A)
{
    extern __shared__ float smem[];
    const FfnnDev &net = A.net;
    const int L = net.n_layers, N = net.widths[0];
    const int S = A.lds_stride;
    float *in0 = smem;                  // [N] spins
    float *z = smem + S;                // [L][S] pre-activations
    float *dl = z + (size_t)L * S;      // [2][S] deltas (ping-pong)
    __shared__ float red[4];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int64_t smp = blockIdx.x; smp < A.n; smp += gridDim.x) {
        for (int i = tid; i < N; i += nt) in0[i] = (float)A.samples[smp * N + i];
        __syncthreads();
        // forward
        for (int l = 0; l < L; ++l) {
            const int out = net.widths[l + 1], in = net.widths[l];
            const float *src = l == 0 ? in0 : z + (size_t)(l - 1) * S;
            const float *Wt = net.Wt[l];
            for (int r = tid; r < out; r += nt) {
                float acc = net.b[l][r];
                if (l == 0) {
                    for (int k = 0; k < in; ++k) acc = fmaf(Wt[(size_t)k * out + r], src[k], acc);
                } else {
                    for (int k = 0; k < in; ++k) acc = fmaf(Wt[(size_t)k * out + r], fmaxf(src[k], 0.0f), acc);
                }
                z[(size_t)l * S + r] = acc;
            }
            __syncthreads();
        }
        // log psi
        const int wl = net.widths[L];
        float part = 0.0f;
        for (int r = tid; r < wl; r += nt) part += logcosh_f32(z[(size_t)(L - 1) * S + r]);
        part = group_sum<64>(part);
        if ((tid & 63) == 0) red[tid >> 6] = part;
        __syncthreads();
        if (tid == 0 && A.logpsi) A.logpsi[smp] = red[0] + red[1] + red[2] + red[3];
        if (A.O) {
            const int64_t p0 = A.p0, p1 = A.p1;
            float *O = A.O + smp * (p1 - p0) - p0;   // O[p] for p in [p0, p1)
            // parameter offsets
            int64_t offW[NQS_MAX_LAYERS], offb[NQS_MAX_LAYERS], off = 0;
            for (int l = 0; l < L; ++l) {
                offW[l] = off;
                off += (int64_t)net.widths[l + 1] * net.widths[l];
                offb[l] = off;
                off += net.widths[l + 1];
            }
            float *d = dl;
            for (int r = tid; r < wl; r += nt) d[r] = tanhf(z[(size_t)(L - 1) * S + r]);
            __syncthreads();
            for (int l = L - 1; l >= 0; --l) {
                const int out = net.widths[l + 1], in = net.widths[l];
                const float *src = l == 0 ? in0 : z + (size_t)(l - 1) * S;
                for (int r = tid; r < out; r += nt)
                    if (offb[l] + r >= p0 && offb[l] + r < p1) O[offb[l] + r] = d[r];
                // O_W[r][k] = d[r] * h[k], consecutive threads on consecutive k; rows
                // [r0, r1) of this layer meet the column range
                const int r0 = (int)min((int64_t)out, max((int64_t)0, (p0 - offW[l]) / in));
                const int r1 = (int)min((int64_t)out, max((int64_t)0, (p1 - offW[l] + in - 1) / in));
                for (int r = r0; r < r1; ++r) {
                    const float dr = d[r];
                    const int64_t rb = offW[l] + (int64_t)r * in;
                    const int k0 = (int)max((int64_t)0, p0 - rb), k1 = (int)min((int64_t)in, p1 - rb);
                    float *orow = O + rb;
                    if (l == 0) {
                        for (int k = k0 + tid; k < k1; k += nt) orow[k] = dr * src[k];
                    } else {
                        for (int k = k0 + tid; k < k1; k += nt) orow[k] = dr * fmaxf(src[k], 0.0f);
                    }
                }
                // parameters of the layers below lie before offW[l]
                if (l == 0 || offW[l] <= p0) break;
                float *dn = (d == dl) ? dl + S : dl;
                const float *W = net.W[l];
                for (int k = tid; k < in; k += nt) {
                    float g = 0.0f;
                    for (int r = 0; r < out; ++r) g = fmaf(W[(size_t)r * in + k], d[r], g);
                    dn[k] = src[k] > 0.0f ? g : 0.0f;
                }
                __syncthreads();
                d = dn;
            }
        }
        __syncthreads();
    }
}

// vjp_out[p] += sum_k g[k] O[k][p] over a chunk of samples (FP64 accumulation per chunk)
__global__ void vjp_chunk_kernel(const float *__restrict__ O, const float *__restrict__ g, int64_t n, int64_t P,
                                 float *__restrict__ out, int first)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    double acc = first ? 0.0 : (double)out[p];
    for (int64_t k = 0; k < n; ++k) acc += (double)g[k] * (double)O[k * P + p];
    out[p] = (float)acc;
}

nqs_status launch_vjp_chunk(const float *O, const float *g, int64_t n, int64_t P, float *out, bool first,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(vjp_chunk_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, O, g, n, P, out,
                       first ? 1 : 0);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// Factors of O for B samples per block: the layer inputs a_{l-1} (post-ReLU) and
// the deltas of every layer.  Each weight read from memory serves B samples;
// per sample the arithmetic (and its order) is that of ffnn_grad_kernel, so
// delta_l[r] * a_{l-1}[c] reproduces its O bit for bit.
template <int B>
__global__ void __launch_bounds__(256) ffnn_factor_kernel(GradArgs A)
{
    extern __shared__ float smem[];
    const FfnnDev &net = A.net;
    const int L = net.n_layers, N = net.widths[0];
    // per sample, packed: spins [N], pre-activations of every layer, two delta vectors of S floats
    const int S = A.lds_stride;
    const int tid = threadIdx.x, nt = blockDim.x;
    int64_t sa = 0, sd = 0;
    int zoff[NQS_MAX_LAYERS];
    int R = (N + 3) & ~3;
    for (int l = 0; l < L; ++l) {
        sa += net.widths[l];
        sd += net.widths[l + 1];
        zoff[l] = R;
        R += (net.widths[l + 1] + 3) & ~3;
    }
    const int doff = R;
    R += 2 * S;
    auto in0 = [&](int b) { return smem + (size_t)b * R; };
    auto zl = [&](int b, int l) { return smem + (size_t)b * R + zoff[l]; };
    auto dlb = [&](int b, int h) { return smem + (size_t)b * R + doff + (size_t)h * S; };
    for (int64_t s0 = (int64_t)blockIdx.x * B; s0 < A.n; s0 += (int64_t)gridDim.x * B) {
        const int nb = (int)min((int64_t)B, A.n - s0);
        for (int e = tid; e < B * N; e += nt) {
            const int b = e / N, i = e - b * N;
            in0(b)[i] = b < nb ? (float)A.samples[(s0 + b) * N + i] : 0.0f;
        }
        __syncthreads();
        for (int l = 0; l < L; ++l) {
            const int out = net.widths[l + 1], in = net.widths[l];
            const float *Wt = net.Wt[l];
            for (int r = tid; r < out; r += nt) {
                float acc[B];
#pragma unroll
                for (int b = 0; b < B; ++b) acc[b] = net.b[l][r];
#pragma unroll 4
                for (int k = 0; k < in; ++k) {
                    const float w = Wt[(size_t)k * out + r];
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const float x = l == 0 ? in0(b)[k] : fmaxf(zl(b, l - 1)[k], 0.0f);
                        acc[b] = fmaf(w, x, acc[b]);
                    }
                }
#pragma unroll
                for (int b = 0; b < B; ++b) zl(b, l)[r] = acc[b];
            }
            __syncthreads();
        }
        // layer inputs
        for (int b = 0; b < nb; ++b) {
            float *ar = A.acts + (s0 + b) * sa;
            int64_t oa = 0;
            for (int l = 0; l < L; ++l) {
                const int in = net.widths[l];
                for (int k = tid; k < in; k += nt) ar[oa + k] = l == 0 ? in0(b)[k] : fmaxf(zl(b, l - 1)[k], 0.0f);
                oa += in;
            }
        }
        const int wl = net.widths[L];
        for (int e = tid; e < B * wl; e += nt) {
            const int b = e / wl, r = e - b * wl;
            dlb(b, 0)[r] = tanhf(zl(b, L - 1)[r]);
        }
        __syncthreads();
        int h = 0;
        int64_t od = sd;
        for (int l = L - 1; l >= 0; --l) {
            const int out = net.widths[l + 1], in = net.widths[l];
            od -= out;
            for (int b = 0; b < nb; ++b) {
                float *dr = A.dels + (s0 + b) * sd + od;
                for (int r = tid; r < out; r += nt) dr[r] = dlb(b, h)[r];
            }
            if (l == 0) break;
            const float *W = net.W[l];
            for (int k = tid; k < in; k += nt) {
                float g[B];
#pragma unroll
                for (int b = 0; b < B; ++b) g[b] = 0.0f;
#pragma unroll 4
                for (int r = 0; r < out; ++r) {
                    const float w = W[(size_t)r * in + k];
#pragma unroll
                    for (int b = 0; b < B; ++b) g[b] = fmaf(w, dlb(b, h)[r], g[b]);
                }
#pragma unroll
                for (int b = 0; b < B; ++b) dlb(b, h ^ 1)[k] = zl(b, l - 1)[k] > 0.0f ? g[b] : 0.0f;
            }
            __syncthreads();
            h ^= 1;
        }
        __syncthreads();
    }
}

nqs_status ffnn_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                            const float *vjp_in, float *vjp_out, hipStream_t stream, int64_t p0, int64_t p1)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const FfnnDev &net = m->copies[NQS_F32].ffnn;
    int maxw = net.widths[0];
    for (int l = 1; l <= net.n_layers; ++l) maxw = std::max(maxw, net.widths[l]);
    GradArgs A;
    A.net = net;
    A.P = m->P;
    A.p0 = p0;
    A.p1 = p1;
    A.acts = nullptr;
    A.dels = nullptr;
    A.lds_stride = (maxw + 3) & ~3;
    const size_t lds = sizeof(float) * (size_t)A.lds_stride * (1 + net.n_layers + 2);
    if (lds > 160 * 1024) return set_error(NQS_EUNSUPPORTED, "network too wide for the gradient kernel");
    allow_lds(ffnn_grad_kernel, lds);
    const int blocks = (int)std::min<int64_t>(n, 4096);
    if (logpsi || O) {
        A.samples = samples;
        A.n = n;
        A.logpsi = logpsi;
        A.O = O;
        hipLaunchKernelGGL(ffnn_grad_kernel, dim3(blocks), dim3(256), lds, stream, A);
        NQS_HIP_TRY(hipGetLastError());
    }
    if (vjp_in) {
        // chunks of samples through a workspace O block
        const int64_t P = m->P;
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(256ll << 20) / (int64_t)(P * 4)));
        float *Ow = (float *)workspace(sizeof(float) * (size_t)chunk * P, stream);
        if (!Ow) return set_error(NQS_ENOMEM, "workspace allocation failed");
        for (int64_t k0 = 0; k0 < n; k0 += chunk) {
            const int64_t kn = std::min(chunk, n - k0);
            A.samples = samples + k0 * net.widths[0];
            A.n = kn;
            A.logpsi = nullptr;
            A.O = Ow;
            A.p0 = 0;
            A.p1 = P;
            hipLaunchKernelGGL(ffnn_grad_kernel, dim3((unsigned)std::min<int64_t>(kn, 4096)), dim3(256), lds, stream, A);
            hipLaunchKernelGGL(vjp_chunk_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, Ow,
                               vjp_in + k0, kn, P, vjp_out, k0 == 0 ? 1 : 0);
            NQS_HIP_TRY(hipGetLastError());
        }
    }
    return NQS_OK;
}

}  // namespace nqs

namespace nqs {

nqs_status ffnn_sample_dispatch(int dtype, int QK, bool trace, const FfnnSampleArgs &A, int blocks, size_t lds,
                                hipStream_t s);
nqs_status ffnn_eloc_dispatch(int dtype, int QK, const FfnnElocArgs &A, int blocks, size_t lds, hipStream_t s);
bool ffnn_reg_sample_launch_bf16(int ke, bool trace, bool perchain, const FfnnSampleArgs &A, int blocks, size_t lds,
                              hipStream_t s);
bool ffnn_reg_sample_launch_f16(int ke, bool trace, bool perchain, const FfnnSampleArgs &A, int blocks, size_t lds,
                              hipStream_t s);
size_t ffnn_reg_sample_lds_bf16(int N, int ke, int m2p);
size_t ffnn_reg_sample_lds_f16(int N, int ke, int m2p);
bool ffnn_reg_eloc_launch_bf16(int ke, const FfnnElocArgs &A, int G, int blocks, size_t lds, hipStream_t s);
bool ffnn_reg_eloc_launch_f16(int ke, const FfnnElocArgs &A, int G, int blocks, size_t lds, hipStream_t s);
size_t ffnn_reg_eloc_lds_bf16(int N, int ke, int m2p, int G);
size_t ffnn_reg_eloc_lds_f16(int N, int ke, int m2p, int G);
// Layer 2 can live in registers (8 waves x 32 output rows) for 16-bit operands
// with 128 <= m1p <= 512 and m2p <= 256.
static_assert(kRows == kRegRows, "both samplers take 64 chains per block");
static bool reg_path(int dtype, const FfnnDev &f)
{
    return (dtype == NQS_BF16 || dtype == NQS_F16) && f.m1p >= 128 && f.m1p <= 512 && f.m2p <= 256;
}

nqs_status deep_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                       uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream);
nqs_status deep_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                             double *eloc, hipStream_t stream);

// Copy ready; *deep tells whether the network goes through the batched-GEMM path
// (any depth) instead of the two-layer kernels with an incremental first layer.
static nqs_status ffnn_mc_ready(nqs_model *m, int dtype, hipStream_t stream, bool *deep)
{
    if (dtype != NQS_F32 && dtype != NQS_BF16 && dtype != NQS_F16 && dtype != NQS_FP8_E4M3)
        return set_error(NQS_EUNSUPPORTED, "dense networks sample in F32, BF16, F16 or FP8_E4M3");
    nqs_status st = ensure_copy(m, dtype, stream);
    if (st != NQS_OK) return st;
    const FfnnDev &f = m->copies[dtype].ffnn;
    // the FP8 copy runs only the batched path (its layer products need whole E4M3 operand tiles)
    *deep = dtype == NQS_FP8_E4M3 || m->desc.n_layers != 2 || f.m1p > 512 ||
            (int64_t)f.widths[0] * f.m1p * (dtype == NQS_F32 ? 0 : 2) > 96 * 1024;
    return NQS_OK;
}

static size_t sample_lds_bytes(int dtype, int N, int m1p, int m2p)
{
    if (dtype == NQS_F32) return FfnnLds<float>::bytes(N, m1p, m2p);
    if (dtype == NQS_F16) return FfnnLds<_Float16>::bytes(N, m1p, m2p);
    return FfnnLds<__bf16>::bytes(N, m1p, m2p);
}

nqs_status ffnn_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                       uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream)
{
    bool deep = false;
    nqs_status st = ffnn_mc_ready(m, cfg.dtype, stream, &deep);
    if (st != NQS_OK) return st;
    if (deep || cfg.lanes_per_chain == -1) {
        if ((int64_t)(cfg.n_burnin + cfg.n_sweeps) * (cfg.sweep_size > 0 ? cfg.sweep_size : m->desc.n_visible) == 0) {
            if (cfg.init_chains) {
                st = launch_init_chains(chain_state, cfg.n_chains, m->desc.n_visible, cfg.move, cfg.seed,
                                        cfg.instance_id, cfg.chain_id_offset, stream);
                if (st != NQS_OK) return st;
            }
            if (n_accepted) return launch_zero_u64(n_accepted, cfg.n_chains, stream);
            return NQS_OK;
        }
        return deep_sample(m, cfg, chain_state, samples, logpsi, n_accepted, trace, stream);
    }
    const FfnnDev &f = m->copies[cfg.dtype].ffnn;
    const int N = f.widths[0];
    const int KE = f.n_layers >= 2 ? (f.widths[1] + 15) / 16 : 0;   // 16-wide fragments multiplied
    const size_t reg_lds = cfg.dtype == NQS_F16 ? ffnn_reg_sample_lds_f16(N, KE, f.m2p) : ffnn_reg_sample_lds_bf16(N, KE, f.m2p);
    const bool use_reg = reg_path(cfg.dtype, f) && reg_lds <= 160 * 1024;
    const size_t lds = use_reg ? reg_lds : sample_lds_bytes(cfg.dtype, N, f.m1p, f.m2p);
    if (lds > 160 * 1024) return set_error(NQS_EUNSUPPORTED, "network too large for the LDS-resident sampler");
    if (cfg.init_chains) {
        st = launch_init_chains(chain_state, cfg.n_chains, N, cfg.move, cfg.seed, cfg.instance_id, cfg.chain_id_offset,
                                stream);
        if (st != NQS_OK) return st;
    }
    FfnnSampleArgs A;
    A.net = f;
    A.W2 = cfg.dtype == NQS_F32 ? (const void *)f.W2p : (const void *)f.W2c;
    A.W1t = cfg.dtype == NQS_F32 ? (const void *)f.W1tp : (const void *)f.W1ct;
    A.chain_state = chain_state;
    A.samples = samples;
    A.logpsi = logpsi;
    A.n_acc = (unsigned long long *)n_accepted;
    A.n_chains = cfg.n_chains;
    A.n_sweeps = cfg.n_sweeps;
    A.n_burnin = cfg.n_burnin;
    A.sweep_size = cfg.sweep_size > 0 ? cfg.sweep_size : N;
    A.refresh_sweeps = cfg.refresh_sweeps > 0 ? cfg.refresh_sweeps : 1;
    A.move = cfg.move;
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
    if ((int64_t)(cfg.n_burnin + cfg.n_sweeps) * A.sweep_size == 0) {
        if (n_accepted) return launch_zero_u64(n_accepted, cfg.n_chains, stream);
        return NQS_OK;
    }
    const int QK = (f.m1p + 63) / 64;
    const int64_t blocks = (cfg.n_chains + kRows - 1) / kRows;   // kRows == kRegRows: 64 chains per block
    if (use_reg) {
        // With exchange moves about half the proposals swap equal spins: chains that
        // advance on their own decide those on the spot and fill every tile with
        // effective rows.  Flip moves are all effective, so the chains step together.
        const bool perchain = A.move == NQS_MOVE_EXCHANGE;
        const bool ok = cfg.dtype == NQS_F16 ? ffnn_reg_sample_launch_f16(KE, tr, perchain, A, (int)blocks, lds, stream)
                                             : ffnn_reg_sample_launch_bf16(KE, tr, perchain, A, (int)blocks, lds, stream);
        if (!ok) return set_error(NQS_EUNSUPPORTED, "first hidden width not supported by the register-resident sampler");
        NQS_HIP_TRY(hipGetLastError());
        return NQS_OK;
    }
    return ffnn_sample_dispatch(cfg.dtype, QK, tr, A, (int)blocks, lds, stream);
}

nqs_status ffnn_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                             double *eloc, hipStream_t stream)
{
    bool deep = false;
    nqs_status st = ffnn_mc_ready(m, dtype, stream, &deep);
    if (st != NQS_OK) return st;
    if (m->desc.marshall && (m->desc.lat_dim != ham.dim || m->desc.lat_L != ham.L))
        return set_error(NQS_EINVAL, "Marshall lattice differs from the Hamiltonian lattice");
    if (deep) return deep_local_energy(m, ham, samples, n, dtype, eloc, stream);
    const FfnnDev &f = m->copies[dtype].ffnn;
    const int N = f.widths[0];
    size_t lds;
    // the register-resident kernel: W1 (16 KE columns) in LDS and groups of G samples, the largest G of 8, 4, 2,
    // 1 whose rows the LDS holds (N < 8191 for the packed row codes)
    const int KE = f.n_layers >= 2 ? (f.widths[1] + 15) / 16 : 0;   // 16-wide fragments multiplied
    auto reg_lds_for = [&](int G) {
        return dtype == NQS_F16 ? ffnn_reg_eloc_lds_f16(N, KE, f.m2p, G) : ffnn_reg_eloc_lds_bf16(N, KE, f.m2p, G);
    };
    int reg_G = 8;
    while (reg_G > 1 && reg_lds_for(reg_G) > 160 * 1024) reg_G /= 2;
    const size_t reg_lds = reg_path(dtype, f) ? reg_lds_for(reg_G) : 0;
    const bool use_reg = reg_path(dtype, f) && reg_lds <= 160 * 1024 && N < 8191;
    if (use_reg) lds = reg_lds;
    else if (dtype == NQS_F32) lds = ffnn_eloc_lds_bytes<float>(N, f.m1p, f.m2p);
    else if (dtype == NQS_F16) lds = ffnn_eloc_lds_bytes<_Float16>(N, f.m1p, f.m2p);
    else lds = ffnn_eloc_lds_bytes<__bf16>(N, f.m1p, f.m2p);
    if (lds > 160 * 1024) return set_error(NQS_EUNSUPPORTED, "network too large for the local-energy kernel");
    if (m->desc.marshall && (m->desc.lat_dim != ham.dim || m->desc.lat_L != ham.L))
        return set_error(NQS_EINVAL, "Marshall lattice differs from the Hamiltonian lattice");
    FfnnElocArgs A;
    A.net = f;
    A.W2 = dtype == NQS_F32 ? (const void *)f.W2p : (const void *)f.W2c;
    A.W1t = dtype == NQS_F32 ? (const void *)f.W1tp : (const void *)f.W1ct;
    A.samples = samples;
    A.n = n;
    A.kind = ham.kind;
    A.dim = ham.dim;
    A.L = ham.L;
    A.pbc = ham.pbc;
    A.marshall = m->desc.marshall;
    A.J = ham.J;
    A.h = ham.h;
    A.eloc = eloc;
    const int QK = (f.m1p + 63) / 64;
    if (use_reg) {
        const int blocks = (int)std::min<int64_t>((n + reg_G - 1) / reg_G, device_cus());
        const bool ok = dtype == NQS_F16 ? ffnn_reg_eloc_launch_f16(KE, A, reg_G, blocks, lds, stream)
                                         : ffnn_reg_eloc_launch_bf16(KE, A, reg_G, blocks, lds, stream);
        if (!ok) return set_error(NQS_EUNSUPPORTED, "first hidden width not supported by the local-energy kernel");
        NQS_HIP_TRY(hipGetLastError());
        return NQS_OK;
    }
    const int blocks = (int)std::min<int64_t>(n, 256 * 4);
    return ffnn_eloc_dispatch(dtype, QK, A, blocks, lds, stream);
}

// ---- sample-space Gram matrix from the factors of O ----
//
// O of a dense layer is an outer product per sample: O_{W_l}[r][c] = delta_l[r] *
// a_{l-1}[c], O_{b_l}[r] = delta_l[r].  The factors (a few thousand floats per
// sample) are computed once; each column block of O is then expanded from them
// (a write-bound pass) instead of rerunning the forward and backward passes.

struct ExpandArgs {
    const float *acts, *dels;
    float *O;                     // [n][p1 - p0]
    int64_t n, p0, p1, sa, sd;    // sa, sd: row lengths of acts and dels
    int L;
    int64_t offW[NQS_MAX_LAYERS + 1];   // first parameter of layer l; offW[L] = P
    int in[NQS_MAX_LAYERS], out[NQS_MAX_LAYERS];
    int64_t offA[NQS_MAX_LAYERS], offD[NQS_MAX_LAYERS];
};

constexpr int kExpandRows = 16;

__global__ void __launch_bounds__(256) ffnn_expand_kernel(ExpandArgs E)
{
    const int64_t p = E.p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= E.p1) return;
    int l = 0;
    while (l + 1 < E.L && p >= E.offW[l + 1]) ++l;
    const int64_t q = p - E.offW[l], nw = (int64_t)E.out[l] * E.in[l];
    int64_t ai, di;
    if (q < nw) {
        const int64_t r = q / E.in[l];
        ai = E.offA[l] + (q - r * E.in[l]);
        di = E.offD[l] + r;
    } else {
        ai = -1;
        di = E.offD[l] + (q - nw);
    }
    const int64_t ldo = E.p1 - E.p0;
    const int64_t k0 = blockIdx.y * (int64_t)kExpandRows, k1 = min(E.n, k0 + kExpandRows);
    for (int64_t k = k0; k < k1; ++k) {
        const float d = E.dels[k * E.sd + di];
        E.O[k * ldo + (p - E.p0)] = ai >= 0 ? d * E.acts[k * E.sa + ai] : d;
    }
}

nqs_status ffnn_factors(nqs_model *m, const int8_t *samples, int64_t n, float *acts, float *dels, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const FfnnDev &net = m->copies[NQS_F32].ffnn;
    const int L = net.n_layers;
    int maxw = net.widths[0];
    for (int l = 1; l <= L; ++l) maxw = std::max(maxw, net.widths[l]);
    GradArgs A;
    A.net = net;
    A.samples = samples;
    A.n = n;
    A.logpsi = nullptr;
    A.O = nullptr;
    A.P = m->P;
    A.p0 = 0;
    A.p1 = m->P;
    A.acts = acts;
    A.dels = dels;
    A.lds_stride = (maxw + 3) & ~3;
    size_t per = (size_t)((net.widths[0] + 3) & ~3) + 2 * (size_t)A.lds_stride;   // LDS floats per sample
    for (int l = 1; l <= L; ++l) per += (size_t)((net.widths[l] + 3) & ~3);
    per *= sizeof(float);
    const int64_t blocks_cap = (int64_t)device_cus() * 16;
    auto launch = [&](auto kernel, int B) {
        allow_lds(kernel, per * B);
        const int64_t blocks = std::min<int64_t>((n + B - 1) / B, blocks_cap);
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), per * B, stream, A);
    };
    // samples per block: each weight read serves B samples, while at least two
    // blocks (eight waves) fit a compute unit's 160 KB of LDS to hide load latency
    if (per * 8 <= 80 * 1024) launch(ffnn_factor_kernel<8>, 8);
    else if (per * 4 <= 80 * 1024) launch(ffnn_factor_kernel<4>, 4);
    else if (per * 2 <= 80 * 1024) launch(ffnn_factor_kernel<2>, 2);
    else if (per <= 160 * 1024) launch(ffnn_factor_kernel<1>, 1);
    else return set_error(NQS_EUNSUPPORTED, "network too wide for the gradient kernel");
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status ffnn_sample_gram(nqs_model *m, const int8_t *samples, int64_t n, int64_t chunk, float *T,
                            hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const FfnnDev &net = m->copies[NQS_F32].ffnn;
    const int L = net.n_layers;
    int maxw = net.widths[0];
    for (int l = 1; l <= L; ++l) maxw = std::max(maxw, net.widths[l]);
    ExpandArgs E;
    E.L = L;
    E.n = n;
    int64_t off = 0, sa = 0, sd = 0;
    for (int l = 0; l < L; ++l) {
        E.in[l] = net.widths[l];
        E.out[l] = net.widths[l + 1];
        E.offW[l] = off;
        off += (int64_t)E.out[l] * E.in[l] + E.out[l];
        E.offA[l] = sa;
        sa += E.in[l];
    }
    E.offW[L] = off;
    for (int l = 0; l < L; ++l) {   // delta_l sits after the deltas of the layers below it
        E.offD[l] = sd;
        sd += E.out[l];
    }
    E.sa = sa;
    E.sd = sd;
    const int64_t P = m->P;
    const size_t fa = (sizeof(float) * (size_t)n * sa + 255) & ~(size_t)255;
    const size_t fd = (sizeof(float) * (size_t)n * sd + 255) & ~(size_t)255;
    const size_t oc = (sizeof(float) * (size_t)n * chunk + 255) & ~(size_t)255;
    char *ws = (char *)workspace(fa + fd + oc + gram_workspace_bytes(n, chunk), stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    float *acts = (float *)ws, *dels = (float *)(ws + fa);
    E.acts = acts;
    E.dels = dels;
    float *Oc = (float *)(ws + fa + fd);

    st = ffnn_factors(m, samples, n, acts, dels, stream);
    if (st != NQS_OK) return st;

    const int64_t ry = (n + kExpandRows - 1) / kExpandRows;
    if (ry > 65535) return set_error(NQS_EINVAL, "too many samples for the expansion grid");
    for (int64_t p0 = 0; p0 < P; p0 += chunk) {
        const int64_t p1 = std::min(P, p0 + chunk);
        E.O = Oc;
        E.p0 = p0;
        E.p1 = p1;
        hipLaunchKernelGGL(ffnn_expand_kernel, dim3((unsigned)((p1 - p0 + 255) / 256), (unsigned)ry), dim3(256), 0,
                           stream, E);
        NQS_HIP_TRY(hipGetLastError());
        st = launch_gram_ws(Oc, n, p1 - p0, p0 == 0 ? 1 : 2, T, ws + fa + fd + oc, stream);
        if (st != NQS_OK) return st;
    }
    return NQS_OK;
}

}  // namespace nqs
