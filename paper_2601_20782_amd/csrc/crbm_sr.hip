// Log-derivatives and the stochastic-reconfiguration step of the
// complex-parameter RBM (App. G with complex a, b, W; App. I.2).
//
// log psi is holomorphic in the complex parameters p = [a, b, W], so
//     O_k = d log psi / d p_k:  s_i (a_i),  tanh theta_j (b_j),  tanh theta_j s_i (W_ji),
// theta = W s + b.  O is stored as [n][2P'] FP32 reals, Re O in the first P'
// columns and Im O in the last P' (the parameter vector's own layout).
//
// SR in sample space with complex parameters: S = Obar^H Obar / n (Eq. eq:smat),
// F = Obar^H (eps - mean eps) / n (Eq. eq:forces), and
//     (S + shift) delta = F  <=>  delta = Obar^H z / n,  (T + shift) z = eps - mean eps,
// with T = Obar Obar^H / n Hermitian (n x n).  T acts on (Re z, Im z) as the
// real 2n x 2n matrix [[Re T, -Im T], [Im T, Re T]], which is the Gram matrix
// of the 2n x 2P' real rows  R = [Re Obar, -Im Obar],  I = [Im Obar, Re Obar]
// (R R^T = I I^T = Re T, I R^T = Im T), so the real Gram kernels and the real
// conjugate-gradient solver apply unchanged.  The update p -> p - lr delta
// moves the real parts by Re delta and the imaginary parts by Im delta.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "crbm_math.h"
#include "internal.h"

namespace nqs {

constexpr int kCrThreads = 256;

static size_t r256(size_t x) { return (x + 255) & ~(size_t)255; }

// theta_j and tanh theta_j of one sample, for j = threadIdx.x, threadIdx.x + blockDim.x, ...
__device__ __forceinline__ float2 crbm_theta(const CrbmDev &net, const float *s, int j)
{
    float2 th = net.b[j];
    for (int i = 0; i < net.N; ++i) {
        const float2 w = net.Wt[(size_t)i * net.M + j];
        th.x = fmaf(w.x, s[i], th.x);
        th.y = fmaf(w.y, s[i], th.y);
    }
    return th;
}

// One block per sample (grid-stride): Re log psi and the row of O.
__global__ void __launch_bounds__(kCrThreads) crbm_grad_kernel(CrbmDev net, const int8_t *__restrict__ samples,
                                                                int64_t n, float *__restrict__ logpsi,
                                                                float *__restrict__ O)
{
    extern __shared__ float sm[];
    const int N = net.N, M = net.M;
    float *s = sm;
    float2 *t = (float2 *)(sm + ((N + 1) & ~1));
    __shared__ float red[kCrThreads / 64];
    const int64_t Pc = (int64_t)N + M + (int64_t)M * N;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) s[i] = (float)samples[q * N + i];
        __syncthreads();
        float lre = 0.0f;
        for (int j = threadIdx.x; j < M; j += blockDim.x) {
            const float2 th = crbm_theta(net, s, j);
            t[j] = ctanh(th);
            lre += clogcosh_re(th);
        }
        for (int i = threadIdx.x; i < N; i += blockDim.x) lre = fmaf(net.a[i].x, s[i], lre);
        if (logpsi) {
            lre = group_sum<64>(lre);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lre;
        }
        __syncthreads();
        if (logpsi && threadIdx.x == 0) {
            float v = 0.0f;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w];
            logpsi[q] = v;
        }
        if (O) {
            float *row = O + q * 2 * Pc;
            for (int64_t k = threadIdx.x; k < Pc; k += blockDim.x) {
                float2 v;
                if (k < N) {
                    v = make_float2(s[k], 0.0f);
                } else if (k < N + M) {
                    v = t[k - N];
                } else {
                    const int64_t kk = k - N - M;
                    const int j = (int)(kk / N), i = (int)(kk - (int64_t)j * N);
                    v = make_float2(t[j].x * s[i], t[j].y * s[i]);
                }
                row[k] = v.x;
                row[Pc + k] = v.y;
            }
        }
        __syncthreads();   // s and t are rewritten by the next sample
    }
}

nqs_status crbm_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                            hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const CrbmDev &net = m->copies[NQS_F32].crbm;
    const size_t lds = sizeof(float) * ((net.N + 1) & ~1) + sizeof(float2) * net.M;
    if (lds > 64 * 1024) return set_error(NQS_EUNSUPPORTED, "complex RBM too large for the log-derivative kernel");
    const int grid = (int)std::min<int64_t>(n, (int64_t)device_cus() * 8);
    hipLaunchKernelGGL(crbm_grad_kernel, dim3(grid), dim3(kCrThreads), lds, stream, net, samples, n, logpsi, O);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// The real embedding of T: Z[2n][2P'] from O[n][2P'], centred per half
// ---------------------------------------------------------------------------
__global__ void cplx_colmean_kernel(const float *__restrict__ O, int64_t n, int64_t cols, double *__restrict__ mu)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double acc = 0.0;
    for (int64_t r = 0; r < n; ++r) acc += (double)O[r * cols + c];
    mu[c] = acc / (double)n;
}

__global__ void cplx_embed_kernel(const float *__restrict__ O, int64_t n, int64_t Pc, const double *__restrict__ mu,
                                  float *__restrict__ Z)
{
    const int64_t cols = 2 * Pc, total = 2 * n * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e - r * cols;
        const int64_t s = r < n ? r : r - n;
        const bool first = c < Pc;
        const int64_t k = first ? c : c - Pc;
        const double re = (double)O[s * cols + k] - mu[k];
        const double im = (double)O[s * cols + Pc + k] - mu[Pc + k];
        double v;
        if (r < n) v = first ? re : -im;   // R = [Re Obar, -Im Obar]
        else v = first ? im : re;          // I = [Im Obar, Re Obar]
        Z[e] = (float)v;
    }
}

__global__ void scale_f32_kernel(float *x, int64_t n, float f)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        x[p] *= f;
}

nqs_status cplx_gram_embedded(const float *O, int64_t n, int64_t P, float *T2, hipStream_t stream)
{
    const int64_t Pc = P / 2;
    const size_t zb = r256(sizeof(float) * (size_t)(2 * n) * (size_t)P), mb = r256(sizeof(double) * (size_t)P);
    char *ws = (char *)workspace_slot(2, zb + mb, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    float *Z = (float *)ws;
    double *mu = (double *)(ws + zb);
    hipLaunchKernelGGL(cplx_colmean_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, O, n, P, mu);
    const int64_t total = 2 * n * P;
    const unsigned eb = (unsigned)std::min<int64_t>((total + 255) / 256, (int64_t)device_cus() * 32);
    hipLaunchKernelGGL(cplx_embed_kernel, dim3(eb), dim3(256), 0, stream, O, n, Pc, (const double *)mu, Z);
    NQS_HIP_TRY(hipGetLastError());
    // the Gram kernel divides by its row count 2n and subtracts the column means of Z (zero up to rounding)
    nqs_status st = launch_gram(Z, 2 * n, P, 1, T2, stream);
    if (st != NQS_OK) return st;
    const int64_t tn = 4 * n * n;
    hipLaunchKernelGGL(scale_f32_kernel, dim3((unsigned)std::min<int64_t>((tn + 255) / 256, (int64_t)device_cus() * 32)),
                       dim3(256), 0, stream, T2, tn, 2.0f);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// Right-hand side of the complex solve: (Re eps - mean, Im eps - mean)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) cplx_rhs_kernel(const double *__restrict__ re, const double *__restrict__ im,
                                                       int64_t n, double *__restrict__ e2)
{
    __shared__ double red[2][4];
    double a = 0.0, b = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x) {
        a += re[s];
        b += im[s];
    }
    a = group_sum<64>(a);
    b = group_sum<64>(b);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    const double ma = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / (double)n;
    const double mb = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / (double)n;
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x) {
        e2[s] = re[s] - ma;
        e2[n + s] = im[s] - mb;
    }
}

nqs_status cplx_sr_rhs(const double *eloc_re, const double *eloc_im, int64_t n, double **e2, hipStream_t stream)
{
    *e2 = (double *)workspace_slot(2, r256(sizeof(double) * 2 * (size_t)n), stream);
    if (!*e2) return set_error(NQS_ENOMEM, "workspace allocation failed");
    hipLaunchKernelGGL(cplx_rhs_kernel, dim3(1), dim3(256), 0, stream, eloc_re, eloc_im, n, *e2);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// Update: master -= lr [Re delta, Im delta],  delta_k = sum_s conj(O_sk) (z_s - mean z) / n
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kCrThreads) crbm_tanh_kernel(CrbmDev net, const int8_t *__restrict__ samples,
                                                                int64_t n, float2 *__restrict__ t)
{
    extern __shared__ float sm[];
    float *s = sm;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        for (int i = threadIdx.x; i < net.N; i += blockDim.x) s[i] = (float)samples[q * net.N + i];
        __syncthreads();
        for (int j = threadIdx.x; j < net.M; j += blockDim.x) t[q * net.M + j] = ctanh(crbm_theta(net, s, j));
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) cplx_zmean_kernel(const double *__restrict__ y, int64_t n, double *__restrict__ zm)
{
    __shared__ double red[2][4];
    double a = 0.0, b = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x) {
        a += y[s];
        b += y[n + s];
    }
    a = group_sum<64>(a);
    b = group_sum<64>(b);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        zm[0] = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / (double)n;
        zm[1] = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / (double)n;
    }
}

__global__ void crbm_update_kernel(int N, int M, const int8_t *__restrict__ samples, const float2 *__restrict__ t,
                                   int64_t n, const double *__restrict__ y, const double *__restrict__ zm, double lr,
                                   double *__restrict__ master)
{
    const int64_t Pc = (int64_t)N + M + (int64_t)M * N;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= Pc) return;
    int kind, i = 0, j = 0;
    if (k < N) {
        kind = 0;
        i = (int)k;
    } else if (k < N + M) {
        kind = 1;
        j = (int)(k - N);
    } else {
        kind = 2;
        const int64_t kk = k - N - M;
        j = (int)(kk / N);
        i = (int)(kk - (int64_t)j * N);
    }
    const double mr = zm[0], mi = zm[1];
    double ar = 0.0, ai = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const double wr = y[s] - mr, wi = y[n + s] - mi;
        double o_r, o_i;   // O_sk
        if (kind == 0) {
            o_r = (double)samples[s * N + i];
            o_i = 0.0;
        } else {
            const float2 tv = t[s * M + j];
            const double sv = kind == 2 ? (double)samples[s * N + i] : 1.0;
            o_r = (double)tv.x * sv;
            o_i = (double)tv.y * sv;
        }
        // conj(O) w
        ar += o_r * wr + o_i * wi;
        ai += o_r * wi - o_i * wr;
    }
    master[k] -= lr * ar / (double)n;
    master[Pc + k] -= lr * ai / (double)n;
}

nqs_status crbm_sr_update(nqs_model *m, const int8_t *samples, int64_t n, const double *y, double lr, double *master,
                          hipStream_t stream)
{
    nqs_status st = ensure_copy(m, NQS_F32, stream);
    if (st != NQS_OK) return st;
    const CrbmDev &net = m->copies[NQS_F32].crbm;
    const size_t tb = r256(sizeof(float2) * (size_t)n * net.M);
    char *ws = (char *)workspace_slot(2, tb + 256, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    float2 *t = (float2 *)ws;
    double *zm = (double *)(ws + tb);
    const size_t lds = sizeof(float) * (size_t)net.N;
    const int grid = (int)std::min<int64_t>(n, (int64_t)device_cus() * 8);
    hipLaunchKernelGGL(crbm_tanh_kernel, dim3(grid), dim3(kCrThreads), lds, stream, net, samples, n, t);
    hipLaunchKernelGGL(cplx_zmean_kernel, dim3(1), dim3(256), 0, stream, y, n, zm);
    const int64_t Pc = (int64_t)net.N + net.M + (int64_t)net.M * net.N;
    hipLaunchKernelGGL(crbm_update_kernel, dim3((unsigned)((Pc + 255) / 256)), dim3(256), 0, stream, net.N, net.M,
                       samples, (const float2 *)t, n, y, (const double *)zm, lr, master);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
