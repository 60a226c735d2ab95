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
//   mix_potrf_kernel   L_kk and D_k = L_kk^{-1} (FP32, one wave, rows in registers)
//   mix_panel_kernel   L_Ik = A_Ik D_k^T for I > k (FP32 matrix cores)
//   mix_update_kernel  A_IJ -= L_Ik L_Jk^T for k < J <= I: the O(n^3) part, on
//                      the matrix cores with operands rounded to the format
//                      (16x16x32 BF16/FP16 or 16x16x4 FP32), FP32 accumulation;
//                      columns outside the current group of four block columns
//                      take the group's four updates in one pass
// then L^{-1} by recursive doubling: with groups of s diagonal tiles inverted,
// adjacent groups join as [[L11, 0], [L21, L22]]^{-1} = [[Linv11, 0],
// [-Linv22 L21 Linv11, Linv22]] (two batched tile products per doubling,
// operands in the format), into B's lower tiles; finally the transpose into
// A's upper tiles (the L tiles there are dead by then), so both triangular
// products of the preconditioner read rows.  Tile operands are staged in LDS.  A pivot that is not larger than the format's
// unit round-off times the original diagonal entry is replaced by that
// entry (counted), which keeps L's diagonal positive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "internal.h"

namespace nqs {

constexpr int kMixNb = 64;
constexpr int kMixGroup = 4;   // block columns per trailing update

typedef short mix_s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 mix_b16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 mix_h16x8 __attribute__((ext_vector_type(8)));
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

constexpr int kMixLd = kMixNb + 4;   // LDS row stride (floats): rows stay 16-byte aligned

// stage a 64 x 64 FP32 tile (row-major, leading dimension ld) into LDS with float4 loads (256 threads)
__device__ __forceinline__ void mix_stage(float (*S)[kMixLd], const float *__restrict__ src, int64_t ld)
{
    for (int e = threadIdx.x; e < kMixNb * kMixNb / 4; e += 256) {
        const int row = e >> 4, c4 = (e & 15) << 2;
        *reinterpret_cast<float4 *>(&S[row][c4]) = *reinterpret_cast<const float4 *>(src + (int64_t)row * ld + c4);
    }
}

// Cholesky of the diagonal tile k and its inverse D_k, one wave.  Lane i keeps
// row i in registers; per column j the pivot comes from lane j (readlane),
// the scaled column goes through LDS (one store, broadcast reads), and every
// lane updates its row.  A single wave needs no barriers: its LDS operations
// complete in issue order.
__global__ void __launch_bounds__(64) mix_potrf_kernel(float *__restrict__ A, int64_t np, int k,
                                                       const float *__restrict__ dg, float eps,
                                                       float *__restrict__ Dinv,
                                                       unsigned long long *__restrict__ nfix)
{
    __shared__ float S[kMixNb][kMixLd];       // L^T: row q of S is column q of L
    __shared__ float R[kMixNb][kMixNb + 1];   // staging for coalesced global access
    __shared__ float col[kMixNb], d0s[kMixNb], rinv[kMixNb];
    const int i = threadIdx.x;
    float *blk = A + (int64_t)k * kMixNb * np + (int64_t)k * kMixNb;
    for (int q = 0; q < kMixNb; ++q) R[q][i] = blk[(int64_t)q * np + i];
    d0s[i] = dg[(int64_t)k * kMixNb + i];
    __syncthreads();
    float r[kMixNb];
#pragma unroll
    for (int m = 0; m < kMixNb; ++m) r[m] = R[i][m];
    unsigned fixes = 0;
#pragma unroll
    for (int j = 0; j < kMixNb; ++j) {
        float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r[j]), j));
        const float d0 = d0s[j];
        const bool fix = !(d > eps * fabsf(d0));   // also catches NaN
        if (fix) d = fabsf(d0) > 0.0f ? fabsf(d0) : 1.0f;
        fixes += fix ? 1u : 0u;
        // hardware reciprocal square root (about 1 ulp): the factor only preconditions the FP64 iteration
        const float ri = __builtin_amdgcn_rsqf(d), l = d * ri;
        const float lij = i > j ? r[j] * ri : (i == j ? l : 0.0f);
        r[j] = lij;
        rinv[j] = ri;
        col[i] = lij;
        __syncthreads();
#pragma unroll
        for (int m = j + 1; m < kMixNb; ++m) r[m] = fmaf(-lij, col[m], r[m]);
    }
    // L (zero above the diagonal) into S as L^T and, through R, back to the tile
#pragma unroll
    for (int m = 0; m < kMixNb; ++m) {
        const float v = m <= i ? r[m] : 0.0f;
        S[m][i] = v;
        R[i][m] = v;
    }
    __syncthreads();
    for (int q = 0; q < kMixNb; ++q) blk[(int64_t)q * np + i] = R[q][i];
    // lane c forms column c of L^{-1}, column-oriented: once x[q] is known, the
    // partial sums of the later rows take x[q] times column q of L
    const int c = i;
    float x[kMixNb];
#pragma unroll
    for (int q = 0; q < kMixNb; ++q) x[q] = q == c ? 1.0f : 0.0f;
#pragma unroll
    for (int q = 0; q < kMixNb; ++q) {
        x[q] *= rinv[q];
#pragma unroll
        for (int qq = q + 1; qq < kMixNb; ++qq) x[qq] = fmaf(-S[q][qq], x[q], x[qq]);
    }
    float *D = Dinv + (int64_t)k * kMixNb * kMixNb;
#pragma unroll
    for (int q = 0; q < kMixNb; ++q) D[q * kMixNb + c] = x[q];   // rows q < c hold 0
    if (i == 0 && fixes) atomicAdd(nfix, (unsigned long long)fixes);
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
// eight values as codes of the format
template <int FMT>
__device__ __forceinline__ mix_s16x8 mix_enc8(const float (&v)[8])
{
    mix_s16x8 r;
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = FMT == kBF16 ? mix_bf16(v[q]) : mix_f16(v[q]);
    return r;
}

// acc[x][y] += sum_{kk < 64} As[32 wm + 16 x + i][kk] Bop[kk][32 wn + 16 y + j] for the
// wave's 32 x 32 quadrant (wm, wn), Bop[kk][j] = BT ? Bs[j][kk] : Bs[kk][j]; operands
// rounded to the format; block (x, y) element [4 (lane / 16) + r][lane % 16] in acc[x][y][r].
// The 16-bit formats use the 32-deep instructions (lane group g = lane / 16 supplies
// k = 8 g .. 8 g + 7 of each 32-step, the same slots for A and B).
template <int FMT, bool BT>
__device__ __forceinline__ void mix_mma_lds(mix_f32x4 (&acc)[2][2], const float (*As)[kMixLd],
                                            const float (*Bs)[kMixLd], int wm, int wn)
{
    const int lane = threadIdx.x & 63, la = lane & 15, lk = lane >> 4;
    if constexpr (FMT == kF32) {
#pragma unroll 4
        for (int k0 = 0; k0 < kMixNb; k0 += 4) {
            float a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = As[32 * wm + 16 * x + la][k0 + lk];
                b[x] = BT ? Bs[32 * wn + 16 * x + la][k0 + lk] : Bs[k0 + lk][32 * wn + 16 * x + la];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int k0 = 0; k0 < kMixNb; k0 += 32) {
            mix_s16x8 a[2], b[2];
            const int kb = k0 + 8 * lk;
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                float av[8], bv[8];
                const float4 a0 = *reinterpret_cast<const float4 *>(&As[32 * wm + 16 * x + la][kb]);
                const float4 a1 = *reinterpret_cast<const float4 *>(&As[32 * wm + 16 * x + la][kb + 4]);
                av[0] = a0.x; av[1] = a0.y; av[2] = a0.z; av[3] = a0.w;
                av[4] = a1.x; av[5] = a1.y; av[6] = a1.z; av[7] = a1.w;
                const int jj = 32 * wn + 16 * x + la;
                if constexpr (BT) {
                    const float4 b0 = *reinterpret_cast<const float4 *>(&Bs[jj][kb]);
                    const float4 b1 = *reinterpret_cast<const float4 *>(&Bs[jj][kb + 4]);
                    bv[0] = b0.x; bv[1] = b0.y; bv[2] = b0.z; bv[3] = b0.w;
                    bv[4] = b1.x; bv[5] = b1.y; bv[6] = b1.z; bv[7] = b1.w;
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) bv[q] = Bs[kb + q][jj];
                }
                a[x] = mix_enc8<FMT>(av);
                b[x] = mix_enc8<FMT>(bv);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    if constexpr (FMT == kBF16)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mix_b16x8, a[x]),
                                                                            __builtin_bit_cast(mix_b16x8, b[y]),
                                                                            acc[x][y], 0, 0, 0);
                    else
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(mix_h16x8, a[x]),
                                                                           __builtin_bit_cast(mix_h16x8, b[y]),
                                                                           acc[x][y], 0, 0, 0);
                }
        }
    }
}

// element (ii, jj) of the workgroup's 64 x 64 output held by this thread: f(ii, jj, value)
template <class F>
__device__ __forceinline__ void mix_store(const mix_f32x4 (&acc)[2][2], int wm, int wn, F f)
{
    const int lane = threadIdx.x & 63, la = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) f(32 * wm + 16 * x + 4 * lk + q, 32 * wn + 16 * y + la, acc[x][y][q]);
}

// L_Ik = A_Ik D_k^T for the block rows I = k + 1 + blockIdx.x (FP32 matrix cores)
__global__ void __launch_bounds__(256) mix_panel_kernel(float *__restrict__ A, int64_t np, int k,
                                                        const float *__restrict__ Dinv)
{
    __shared__ float As[kMixNb][kMixLd];
    __shared__ float Ds[kMixNb][kMixLd];
    const int I = k + 1 + blockIdx.x;
    float *blk = A + (int64_t)I * kMixNb * np + (int64_t)k * kMixNb;
    mix_stage(As, blk, np);
    mix_stage(Ds, Dinv + (int64_t)k * kMixNb * kMixNb, kMixNb);
    __syncthreads();
    const int wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
    mix_f32x4 acc[2][2] = {};
    mix_mma_lds<kF32, true>(acc, As, Ds, wm, wn);
    mix_store(acc, wm, wn, [&](int ii, int jj, float v) { blk[(int64_t)ii * np + jj] = v; });
}

// lower-triangular tile pair t -> (r, c), r >= c, t = r (r + 1) / 2 + c
__device__ __forceinline__ void mix_tri(int t, int &r, int &c)
{
    r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    c = t - r * (r + 1) / 2;
}

// A_IJ -= sum_{k0 <= k < k1} L_Ik L_Jk^T over the tiles J = j0 + blockIdx.y,
// I = J + blockIdx.x < nblk (one 64 x 64 tile per workgroup)
template <int FMT>
__global__ void __launch_bounds__(256) mix_update_kernel(float *__restrict__ A, int64_t np, int nblk, int k0, int k1,
                                                         int j0)
{
    __shared__ float As[kMixNb][kMixLd];
    __shared__ float Bs[kMixNb][kMixLd];
    const int J = j0 + blockIdx.y, I = J + blockIdx.x;
    if (I >= nblk) return;
    const int wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
    mix_f32x4 acc[2][2] = {};
    for (int k = k0; k < k1; ++k) {
        mix_stage(As, A + (int64_t)I * kMixNb * np + (int64_t)k * kMixNb, np);
        mix_stage(Bs, A + (int64_t)J * kMixNb * np + (int64_t)k * kMixNb, np);
        __syncthreads();
        mix_mma_lds<FMT, true>(acc, As, Bs, wm, wn);
        __syncthreads();
    }
    float *C = A + (int64_t)I * kMixNb * np + (int64_t)J * kMixNb;
    mix_store(acc, wm, wn, [&](int ii, int jj, float v) { C[(int64_t)ii * np + jj] -= v; });
}

// Inverse of L by recursive doubling.  Groups of s diagonal tiles are already
// inverted (tiles of Linv in B's lower part); pair p joins group 2p (tiles
// [g1, g1 + s)) and group 2p + 1 (tiles [g2, g2 + s2), g2 = g1 + s):
//   X = L21 Linv11,   Linv21 = -Linv22 X,
// X kept transposed in B's upper tiles (g1 + j, g2 + i), unused otherwise.
__global__ void mix_inv_diag_kernel(float *__restrict__ B, int64_t np, const float *__restrict__ Dinv)
{
    const int I = blockIdx.x;
    const float *D = Dinv + (int64_t)I * kMixNb * kMixNb;
    float *dst = B + (int64_t)I * kMixNb * np + (int64_t)I * kMixNb;
    for (int e = threadIdx.x; e < kMixNb * kMixNb; e += blockDim.x) dst[(int64_t)(e >> 6) * np + (e & 63)] = D[e];
}

template <int FMT>
__global__ void __launch_bounds__(256) mix_inv_x_kernel(const float *__restrict__ A, float *__restrict__ B,
                                                        int64_t np, int nblk, int s)
{
    __shared__ float As[kMixNb][kMixLd];
    __shared__ float Bs[kMixNb][kMixLd];
    const int g1 = 2 * s * blockIdx.y, g2 = g1 + s;
    const int s2 = min(s, nblk - g2);
    const int i = blockIdx.x / s, j = blockIdx.x - i * s;
    if (i >= s2) return;
    const int wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
    mix_f32x4 acc[2][2] = {};
    for (int kk = j; kk < s; ++kk) {   // Linv11 is lower triangular: tile (kk, j) with kk >= j
        mix_stage(As, A + (int64_t)(g2 + i) * kMixNb * np + (int64_t)(g1 + kk) * kMixNb, np);
        mix_stage(Bs, B + (int64_t)(g1 + kk) * kMixNb * np + (int64_t)(g1 + j) * kMixNb, np);
        __syncthreads();
        mix_mma_lds<FMT, false>(acc, As, Bs, wm, wn);
        __syncthreads();
    }
    float *Xt = B + (int64_t)(g1 + j) * kMixNb * np + (int64_t)(g2 + i) * kMixNb;
    mix_store(acc, wm, wn, [&](int ii, int jj, float v) { Xt[(int64_t)jj * np + ii] = v; });
}

template <int FMT>
__global__ void __launch_bounds__(256) mix_inv_l_kernel(float *__restrict__ B, int64_t np, int nblk, int s)
{
    __shared__ float As[kMixNb][kMixLd];
    __shared__ float Bs[kMixNb][kMixLd];
    const int g1 = 2 * s * blockIdx.y, g2 = g1 + s;
    const int s2 = min(s, nblk - g2);
    const int i = blockIdx.x / s, j = blockIdx.x - i * s;
    if (i >= s2) return;
    const int wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
    mix_f32x4 acc[2][2] = {};
    for (int kk = 0; kk <= i; ++kk) {   // Linv22 tile (i, kk), X tile (kk, j) stored transposed
        mix_stage(As, B + (int64_t)(g2 + i) * kMixNb * np + (int64_t)(g2 + kk) * kMixNb, np);
        mix_stage(Bs, B + (int64_t)(g1 + j) * kMixNb * np + (int64_t)(g2 + kk) * kMixNb, np);
        __syncthreads();
        mix_mma_lds<FMT, true>(acc, As, Bs, wm, wn);
        __syncthreads();
    }
    float *C = B + (int64_t)(g2 + i) * kMixNb * np + (int64_t)(g1 + j) * kMixNb;
    mix_store(acc, wm, wn, [&](int ii, int jj, float v) { C[(int64_t)ii * np + jj] = -v; });
}

// A's upper tiles (J, I), J <= I, <- the transpose of B's lower tiles (I, J)
__global__ void __launch_bounds__(256) mix_transpose_kernel(const float *__restrict__ B, float *__restrict__ A,
                                                            int64_t np)
{
    __shared__ float S[kMixNb][kMixNb + 1];
    int I, J;
    mix_tri(blockIdx.x, I, J);
    const float *src = B + (int64_t)I * kMixNb * np + (int64_t)J * kMixNb;
    float *dst = A + (int64_t)J * kMixNb * np + (int64_t)I * kMixNb;
    for (int e = threadIdx.x; e < kMixNb * kMixNb; e += 256) S[e >> 6][e & 63] = src[(int64_t)(e >> 6) * np + (e & 63)];
    __syncthreads();
    for (int e = threadIdx.x; e < kMixNb * kMixNb; e += 256) dst[(int64_t)(e >> 6) * np + (e & 63)] = S[e & 63][e >> 6];
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
    // block columns in groups of kMixGroup: inside a group the columns are
    // updated one block column at a time; the trailing matrix takes one
    // rank-(64 x group) update per group, so it is read and written once per
    // group instead of once per block column
    for (int g0 = 0; g0 < nblk; g0 += kMixGroup) {
        const int g1 = min(g0 + kMixGroup, nblk);
        for (int k = g0; k < g1; ++k) {
            hipLaunchKernelGGL(mix_potrf_kernel, dim3(1), dim3(64), 0, s, A, np, k, dg, eps, Dinv, nfix);
            const int rest = nblk - 1 - k;
            if (rest == 0) break;
            hipLaunchKernelGGL(mix_panel_kernel, dim3(rest), dim3(256), 0, s, A, np, k, (const float *)Dinv);
            if (k + 1 < g1)   // columns k + 1 .. g1 - 1 of the group, every row below
                hipLaunchKernelGGL(mix_update_kernel<FMT>, dim3(rest, g1 - k - 1), dim3(256), 0, s, A, np, nblk, k,
                                   k + 1, k + 1);
        }
        if (g1 < nblk)
            hipLaunchKernelGGL(mix_update_kernel<FMT>, dim3(nblk - g1, nblk - g1), dim3(256), 0, s, A, np, nblk, g0,
                               g1, g1);
    }
    hipLaunchKernelGGL(mix_inv_diag_kernel, dim3(nblk), dim3(256), 0, s, B, np, (const float *)Dinv);
    for (int sz = 1; sz < nblk; sz *= 2) {
        const int pairs = (nblk - sz + 2 * sz - 1) / (2 * sz);   // pairs whose second group is not empty
        hipLaunchKernelGGL(mix_inv_x_kernel<FMT>, dim3(sz * sz, pairs), dim3(256), 0, s, (const float *)A, B, np,
                           nblk, sz);
        hipLaunchKernelGGL(mix_inv_l_kernel<FMT>, dim3(sz * sz, pairs), dim3(256), 0, s, B, np, nblk, sz);
    }
    hipLaunchKernelGGL(mix_transpose_kernel, dim3(nblk * (nblk + 1) / 2), dim3(256), 0, s, (const float *)B, A, np);
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
