// Centred Gram matrices of the log-derivatives on FP32 matrix cores:
//   mode 0:  S = Obar^T Obar / n   (Eq. eq:smat, P x P)
//   mode 1:  T = Obar Obar^T / n   (n x n; same non-zero spectrum as S)
// with Obar = O - (column means over samples).  One 128 x 128 output tile per
// block of four waves; each wave owns a 64 x 64 quadrant as 2 x 2
// v_mfma_f32_32x32x2f32 tiles.  The centring is applied while staging tiles
// into LDS, so Obar is never written to memory.  Only tiles on or above the
// block diagonal are computed; the mirror tile is written from the same
// registers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace nqs {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128, kBK = 16;

__global__ void colmean_kernel(const float *__restrict__ O, int64_t n, int64_t P, float *__restrict__ mu)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += (double)O[k * P + p];
    mu[p] = (float)(s / (double)n);
}

// Operand access: element (m, k) of the centred matrix that plays "A" (and "B").
//   TMODE (T = Obar Obar^T): A(m,k) = O[m][k] - mu[k]; m < n, k < P
//   SMODE (S = Obar^T Obar): A(m,k) = O[k][m] - mu[m]; m < P, k < n
template <bool TMODE>
__global__ void __launch_bounds__(256) gram_kernel(const float *__restrict__ O, const float *__restrict__ mu,
                                                   int64_t n, int64_t P, float alpha, float *__restrict__ out)
{
    const int64_t Mdim = TMODE ? n : P;   // output side
    const int64_t Kdim = TMODE ? P : n;   // contraction length
    // map the linear block id onto the upper triangle of tiles (bi <= bj)
    const int64_t nt = (Mdim + kBM - 1) / kBM;
    int64_t t = blockIdx.x, bi = 0;
    while (t >= nt - bi) {
        t -= nt - bi;
        ++bi;
    }
    const int64_t bj = bi + t;
    const int64_t m0 = bi * kBM, n0 = bj * kBM;

    __shared__ float As[kBK][kBM];
    __shared__ float Bs[kBK][kBM];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    floatx16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    for (int64_t k0 = 0; k0 < Kdim; k0 += kBK) {
        // stage 128 x 16 elements of each operand (8 per thread)
        if constexpr (TMODE) {
            const int r = tid >> 1, kh = (tid & 1) * 8;
#pragma unroll
            for (int which = 0; which < 2; ++which) {
                const int64_t row = (which == 0 ? m0 : n0) + r;
                float v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int64_t k = k0 + kh + q;
                    v[q] = (row < Mdim && k < Kdim) ? O[row * P + k] - mu[k] : 0.0f;
                }
                float(*dst)[kBM] = which == 0 ? As : Bs;
#pragma unroll
                for (int q = 0; q < 8; ++q) dst[kh + q][r] = v[q];
            }
        } else {
            const int c = tid & 127, kh = (tid >> 7) * 8;
#pragma unroll
            for (int which = 0; which < 2; ++which) {
                const int64_t col = (which == 0 ? m0 : n0) + c;
                const float muc = col < Mdim ? mu[col] : 0.0f;
                float(*dst)[kBM] = which == 0 ? As : Bs;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int64_t k = k0 + kh + q;
                    dst[kh + q][c] = (col < Mdim && k < Kdim) ? O[k * P + col] - muc : 0.0f;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 2) {
            const int kq = kk + (lane >> 5);
            const float a0 = As[kq][wm + (lane & 31)];
            const float a1 = As[kq][wm + 32 + (lane & 31)];
            const float b0 = Bs[kq][wn + (lane & 31)];
            const float b1 = Bs[kq][wn + 32 + (lane & 31)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    // D[i][j] of a 32x32 tile: lane = j + 32*((i/4)%2), register = i%4 + 4*(i/8)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = lane & 31;
                const int64_t gi = m0 + wm + 32 * a + i, gj = n0 + wn + 32 * b + j;
                const float v = alpha * acc[a][b][r];
                if (gi < Mdim && gj < Mdim) {
                    out[gi * Mdim + gj] = v;
                    if (bi != bj) out[gj * Mdim + gi] = v;
                }
            }
}

nqs_status launch_gram(const float *O, int64_t n, int64_t P, int mode, float *out, hipStream_t stream)
{
    float *mu = (float *)workspace(sizeof(float) * (size_t)P, stream);
    if (!mu) return set_error(NQS_ENOMEM, "workspace allocation failed");
    hipLaunchKernelGGL(colmean_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, O, n, P, mu);
    const int64_t side = mode == 1 ? n : P;
    const int64_t nt = (side + kBM - 1) / kBM;
    const int64_t tiles = nt * (nt + 1) / 2;
    if (tiles > INT32_MAX) return set_error(NQS_EINVAL, "Gram matrix too large");
    const float alpha = (float)(1.0 / (double)n);
    if (mode == 1)
        hipLaunchKernelGGL((gram_kernel<true>), dim3((unsigned)tiles), dim3(256), 0, stream, O, mu, n, P, alpha, out);
    else
        hipLaunchKernelGGL((gram_kernel<false>), dim3((unsigned)tiles), dim3(256), 0, stream, O, mu, n, P, alpha, out);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
