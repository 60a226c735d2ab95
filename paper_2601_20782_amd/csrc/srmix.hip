// Low-precision Cholesky factor of (T + shift) and its inverse, the
// preconditioner of the mixed-precision stochastic-reconfiguration solve.
//
// The system (T + shift) y = e (App. I.2 in sample space) is solved in FP64 by
// conjugate gradients preconditioned with M^{-1} = L^{-T} L^{-1}, where L is a
// Cholesky factor of T + shift computed in a reduced format: the pattern of
// mixed-precision iterative solvers (factorise cheaply, refine in high
// precision) that the paper points to for the preconditioning step (Sec. V),
// in its symmetric positive definite form.  Whatever the factor's rounding,
// M is symmetric positive definite (a triangular factor with positive
// diagonal), so the FP64 iteration converges to the FP64 solution; the
// format only changes the iteration count.
//
// Layout: A = T + shift I padded to np = 64 * ceil(n / 64) rows with an
// identity block (the factor and inverse of the padded matrix are those of
// T + shift, extended by the identity), FP32 row-major with leading
// dimension np, in 64 x 64 tiles.  Blocked right-looking Cholesky, per block
// column k:
//   mix_potrf_kernel   one wave: L_kk and D_k = L_kk^{-1} (FP32, registers + LDS)
//   mix_panel_kernel   L_Ik = A_Ik D_k^T for I > k (FP32)
//   mix_update_kernel  A_IJ -= L_Ik L_Jk^T for k < J <= I: the O(n^3) part, on
//                      the matrix cores with operands rounded to the format
//                      (16x16x16 BF16/FP16 or 16x16x4 FP32), FP32 accumulation
// then the inverse row by row (mix_linv_kernel):
//   Linv_II = D_I,  Linv_IJ = -D_I sum_{K=J}^{I-1} L_IK Linv_KJ   (J < I)
// written to B (lower tiles) and transposed into A's upper tiles (the L
// tiles there are dead by then), so both triangular products of the
// preconditioner read rows.  A pivot that is not larger than the format's
// unit round-off times the original diagonal entry is replaced by that
// entry (counted), which keeps L's diagonal positive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "internal.h"

namespace nqs {

constexpr int kMixNb = 64;

typedef short mix_s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 mix_h16x4 __attribute__((ext_vector_type(4)));
typedef float mix_f32x4 __attribute__((ext_vector_type(4)));

// A = T + shift I, padded with the identity; dg = the diagonal of A
__global__ void mix_build_kernel(const float *__restrict__ T, int64_t n, int64_t np, double shift,
                                 float *__restrict__ A, float *__restrict__ dg)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= np * np) return;
    const int64_t i = idx / np, j = idx - i * np;
    float v;
    if (i < n && j < n) v = i == j ? (float)((double)T[i * n + j] + shift) : T[i * n + j];
    else v = i == j ? 1.0f : 0.0f;
    A[idx] = v;
    if (i == j) dg[i] = v;
}

// Cholesky of the diagonal tile k (one wave, lane i holds row i) and its inverse
__global__ void __launch_bounds__(64) mix_potrf_kernel(float *__restrict__ A, int64_t np, int k,
                                                       const float *__restrict__ dg, float eps,
                                                       float *__restrict__ Dinv,
                                                       unsigned long long *__restrict__ nfix)
{
    __shared__ float col[kMixNb];
    __shared__ float Ls[kMixNb][kMixNb + 1];
    const int i = threadIdx.x;
    float *blk = A + (int64_t)k * kMixNb * np + (int64_t)k * kMixNb;
    float r[kMixNb];
#pragma unroll
    for (int m = 0; m < kMixNb; ++m) r[m] = blk[(int64_t)i * np + m];
    unsigned fixes = 0;
#pragma unroll
    for (int j = 0; j < kMixNb; ++j) {
        float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r[j]), j));
        const float d0 = dg[(int64_t)k * kMixNb + j];
        if (!(d > eps * fabsf(d0))) {   // also catches NaN
            d = fabsf(d0) > 0.0f ? fabsf(d0) : 1.0f;
            ++fixes;
        }
        const float ljj = sqrtf(d);
        const float lij = i == j ? ljj : r[j] / ljj;
        r[j] = lij;
        col[i] = lij;
        __syncthreads();
#pragma unroll
        for (int m = j + 1; m < kMixNb; ++m) r[m] = fmaf(-lij, col[m], r[m]);
        __syncthreads();
    }
    // L into LDS (lower part), then lane c forms column c of L^{-1} by forward substitution
#pragma unroll
    for (int m = 0; m < kMixNb; ++m) Ls[i][m] = m <= i ? r[m] : 0.0f;
    __syncthreads();
    const int c = i;
    float x[kMixNb];
#pragma unroll
    for (int q = 0; q < kMixNb; ++q) {
        float s = q == c ? 1.0f : 0.0f;
#pragma unroll
        for (int m = 0; m < q; ++m) s = fmaf(-Ls[q][m], x[m], s);
        x[q] = s / Ls[q][q];
    }
    float *D = Dinv + (int64_t)k * kMixNb * kMixNb;
#pragma unroll
    for (int q = 0; q < kMixNb; ++q) D[q * kMixNb + c] = x[q];   // rows q < c hold 0
    // L_kk back into A (lower triangle, zero above), coalesced along rows
    for (int q = 0; q < kMixNb; ++q) blk[(int64_t)q * np + i] = Ls[q][i];
    if (i == 0 && fixes) atomicAdd(nfix, (unsigned long long)fixes);
}

// L_Ik = A_Ik D_k^T for the block rows I = k + 1 + blockIdx.x (FP32)
__global__ void __launch_bounds__(256) mix_panel_kernel(float *__restrict__ A, int64_t np, int k,
                                                        const float *__restrict__ Dinv)
{
    __shared__ float As[kMixNb][kMixNb + 1];
    __shared__ float Ds[kMixNb][kMixNb + 1];
    const int I = k + 1 + blockIdx.x;
    float *blk = A + (int64_t)I * kMixNb * np + (int64_t)k * kMixNb;
    const float *D = Dinv + (int64_t)k * kMixNb * kMixNb;
    for (int e = threadIdx.x; e < kMixNb * kMixNb; e += 256) {
        const int q = e >> 6, m = e & 63;
        As[q][m] = blk[(int64_t)q * np + m];
        Ds[q][m] = D[e];
    }
    __syncthreads();
    // out[q][c] = sum_{m <= c} A[q][m] D[c][m]; thread: column c, rows q = rg, rg + 4, ...
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    float acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.0f;
    for (int m = 0; m <= c; ++m) {
        const float dv = Ds[c][m];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = fmaf(As[rg + 4 * t][m], dv, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) blk[(int64_t)(rg + 4 * t) * np + c] = acc[t];
}

// round-to-nearest-even codes of the 16-bit formats
__device__ __forceinline__ short mix_bf16(float v)
{
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ short mix_f16(float v)
{
    const _Float16 h = (_Float16)v;
    return __builtin_bit_cast(short, h);
}

// acc[x][y] (16 x 16 blocks x, y of the wave's 32 x 32 quadrant) += sum over
// kd of fa(i, kk) fb(kk, j), operands rounded to the format; block (x, y)
// element [4 (lane / 16) + r][lane % 16] sits in acc[x][y][r].
template <int FMT, class FA, class FB>
__device__ __forceinline__ void mix_mma(mix_f32x4 (&acc)[2][2], int kd, FA fa, FB fb)
{
    const int lane = threadIdx.x & 63, la = lane & 15, lk = lane >> 4;
    if constexpr (FMT == kF32) {
        for (int k0 = 0; k0 < kd; k0 += 4) {
            float a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = fa(16 * x + la, k0 + lk);
                b[x] = fb(k0 + lk, 16 * x + la);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    } else {
        for (int k0 = 0; k0 < kd; k0 += 16) {
            mix_s16x4 a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float av = fa(16 * x + la, k0 + 4 * lk + q), bv = fb(k0 + 4 * lk + q, 16 * x + la);
                    a[x][q] = FMT == kBF16 ? mix_bf16(av) : mix_f16(av);
                    b[x][q] = FMT == kBF16 ? mix_bf16(bv) : mix_f16(bv);
                }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    if constexpr (FMT == kBF16)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[x], b[y], acc[x][y], 0, 0, 0);
                    else
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(mix_h16x4, a[x]),
                                                                          __builtin_bit_cast(mix_h16x4, b[y]),
                                                                          acc[x][y], 0, 0, 0);
                }
        }
    }
}

// lower-triangular tile pair t -> (r, c), r >= c, t = r (r + 1) / 2 + c
__device__ __forceinline__ void mix_tri(int t, int &r, int &c)
{
    r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    c = t - r * (r + 1) / 2;
}

// A_IJ -= L_Ik L_Jk^T for k < J <= I (one 64 x 64 tile per workgroup, 4 waves)
template <int FMT>
__global__ void __launch_bounds__(256) mix_update_kernel(float *__restrict__ A, int64_t np, int k)
{
    int r, c;
    mix_tri(blockIdx.x, r, c);
    const int I = k + 1 + r, J = k + 1 + c;
    const int wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
    const float *Li = A + ((int64_t)I * kMixNb + 32 * wm) * np + (int64_t)k * kMixNb;
    const float *Lj = A + ((int64_t)J * kMixNb + 32 * wn) * np + (int64_t)k * kMixNb;
    mix_f32x4 acc[2][2] = {};
    mix_mma<FMT>(acc, kMixNb, [&](int i, int kk) { return Li[(int64_t)i * np + kk]; },
                 [&](int kk, int j) { return Lj[(int64_t)j * np + kk]; });
    const int lane = threadIdx.x & 63, la = lane & 15, lk = lane >> 4;
    float *C = A + ((int64_t)I * kMixNb + 32 * wm) * np + (int64_t)J * kMixNb + 32 * wn;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float *dst = C + (int64_t)(16 * x + 4 * lk + q) * np + 16 * y + la;
                *dst -= acc[x][y][q];
            }
}

// block row I of L^{-1}: workgroup J (0 <= J <= I) forms Linv_IJ, stores it
// into B and its transpose into A's tile (J, I)
template <int FMT>
__global__ void __launch_bounds__(256) mix_linv_kernel(float *__restrict__ A, float *__restrict__ B, int64_t np,
                                                       int I, const float *__restrict__ Dinv)
{
    __shared__ float Xs[kMixNb][kMixNb + 1];
    const int J = blockIdx.x;
    const float *D = Dinv + (int64_t)I * kMixNb * kMixNb;
    const int wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
    const int lane = threadIdx.x & 63, la = lane & 15, lk = lane >> 4;
    float *Bt = B + (int64_t)I * kMixNb * np + (int64_t)J * kMixNb;     // Linv_IJ
    float *At = A + (int64_t)J * kMixNb * np + (int64_t)I * kMixNb;     // Linv_IJ^T
    if (J == I) {
        for (int e = threadIdx.x; e < kMixNb * kMixNb; e += 256) {
            const int q = e >> 6, m = e & 63;
            Bt[(int64_t)q * np + m] = D[e];
            At[(int64_t)m * np + q] = D[e];
        }
        return;
    }
    // X = sum_{K=J}^{I-1} L_IK Linv_KJ
    mix_f32x4 acc[2][2] = {};
    for (int K = J; K < I; ++K) {
        const float *Lik = A + ((int64_t)I * kMixNb + 32 * wm) * np + (int64_t)K * kMixNb;
        const float *Lkj = B + (int64_t)K * kMixNb * np + (int64_t)J * kMixNb + 32 * wn;
        mix_mma<FMT>(acc, kMixNb, [&](int i, int kk) { return Lik[(int64_t)i * np + kk]; },
                     [&](int kk, int j) { return Lkj[(int64_t)kk * np + j]; });
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) Xs[32 * wm + 16 * x + 4 * lk + q][32 * wn + 16 * y + la] = acc[x][y][q];
    __syncthreads();
    // Linv_IJ = -D_I X
    mix_f32x4 out[2][2] = {};
    const float *Dw = D + (int64_t)(32 * wm) * kMixNb;
    mix_mma<FMT>(out, kMixNb, [&](int i, int kk) { return Dw[i * kMixNb + kk]; },
                 [&](int kk, int j) { return Xs[kk][32 * wn + j]; });
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = 32 * wm + 16 * x + 4 * lk + q, jj = 32 * wn + 16 * y + la;
                Bt[(int64_t)ii * np + jj] = -out[x][y][q];
                At[(int64_t)jj * np + ii] = -out[x][y][q];
            }
}

size_t mix_workspace_bytes(int64_t n)
{
    const int64_t np = (n + kMixNb - 1) / kMixNb * kMixNb;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return 2 * al(sizeof(float) * (size_t)np * np) + al(sizeof(float) * (size_t)np * kMixNb) +
           al(sizeof(float) * (size_t)np) + 256;
}

template <int FMT>
static void mix_factor_fmt(int64_t np, int nblk, float *A, float *B, float *Dinv, const float *dg, float eps,
                           unsigned long long *nfix, hipStream_t s)
{
    for (int k = 0; k < nblk; ++k) {
        hipLaunchKernelGGL(mix_potrf_kernel, dim3(1), dim3(64), 0, s, A, np, k, dg, eps, Dinv, nfix);
        const int rest = nblk - 1 - k;
        if (rest > 0) {
            hipLaunchKernelGGL(mix_panel_kernel, dim3(rest), dim3(256), 0, s, A, np, k, (const float *)Dinv);
            hipLaunchKernelGGL(mix_update_kernel<FMT>, dim3(rest * (rest + 1) / 2), dim3(256), 0, s, A, np, k);
        }
    }
    for (int I = 0; I < nblk; ++I)
        hipLaunchKernelGGL(mix_linv_kernel<FMT>, dim3(I + 1), dim3(256), 0, s, A, B, np, I, (const float *)Dinv);
}

// Factor and invert: on return Lin (np x np) holds L^{-1} in its lower tiles and
// LinT (np x np) holds L^{-T} in its upper tiles; *nfix (device) counts replaced pivots.
nqs_status mix_factor(const float *T, int64_t n, double shift, int fmt, void *ws, float **Lin, float **LinT,
                      int64_t *np_out, unsigned long long *nfix, hipStream_t s)
{
    const int64_t np = (n + kMixNb - 1) / kMixNb * kMixNb;
    const int nblk = (int)(np / kMixNb);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *p = (char *)ws;
    float *A = (float *)p;
    p += al(sizeof(float) * (size_t)np * np);
    float *B = (float *)p;
    p += al(sizeof(float) * (size_t)np * np);
    float *Dinv = (float *)p;
    p += al(sizeof(float) * (size_t)np * kMixNb);
    float *dg = (float *)p;
    const float eps = fmt == NQS_BF16 ? 0x1p-8f : (fmt == NQS_F16 ? 0x1p-11f : 0x1p-24f);
    const int64_t tot = np * np;
    hipLaunchKernelGGL(mix_build_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, T, n, np, shift, A, dg);
    switch (fmt) {
    case NQS_BF16: mix_factor_fmt<kBF16>(np, nblk, A, B, Dinv, dg, eps, nfix, s); break;
    case NQS_F16: mix_factor_fmt<kF16>(np, nblk, A, B, Dinv, dg, eps, nfix, s); break;
    default: mix_factor_fmt<kF32>(np, nblk, A, B, Dinv, dg, eps, nfix, s); break;
    }
    NQS_HIP_TRY(hipGetLastError());
    *Lin = B;
    *LinT = A;
    *np_out = np;
    return NQS_OK;
}

}  // namespace nqs
