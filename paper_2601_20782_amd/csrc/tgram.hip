// Sample-space Gram matrix T = Obar Obar^T / n (Eq. eq:smat taken in sample
// space, Obar = O - mean over samples) from the factors of O, in FP64.
//
// For every network here a sample's O is a set of outer products: a dense
// layer l gives O_{W_l} = delta_l (x) a_{l-1} and O_{b_l} = delta_l; an RBM gives
// O_W = tanh(theta) (x) s, O_b = tanh(theta), O_a = s.  Writing each layer as a
// pair of per-sample factors U (rows) and V (columns), and c = 1 when V is
// also a block of O on its own (the RBM's visible bias), the dot product of
// two samples' O is
//     K_kl = sum_layers (U_k.U_l + c) (V_k.V_l + 1) - c,
// so K needs Gram matrices of the factors (contractions over a few thousand
// values) instead of one over all P parameters.  Centring is exact algebra:
//     T_kl = (K_kl - v_k - v_l + |mu|^2) / n,   v_k = O_k . mu,
// with mu = mean of O, which per layer is the matrix (1/n) [U,1]^T [V,1]
// (masked to the blocks that exist).  Means, v and K are FP64 throughout
// (products of FP32 factors are exact in FP64); T is rounded to FP32 once.
//
// Kernels: fac_mean (tiled FP64, one block per 64 x 64 tile of a layer's mean
// matrix and range of samples; the ranges summed in order by fac_mean_reduce), fac_v (tiled FP64, per-sample bilinear forms, partials per row
// tile summed in fixed order), fac_gram (FP64 matrix cores,
// v_mfma_f64_16x16x4f64, one block per 64 x 64 tile of T's upper triangle).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace nqs {

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct FacLayer {
    const float *U;   // [n][ldu], first du columns used
    const float *V;   // [n][ldv], first dv columns used
    int64_t ldu, ldv;
    int du, dv;
    int c;            // 1: V is also a block of O by itself
    double *M;        // [(du + 1) x (dv + 1)] masked mean matrix (inside FacArgs::Mall)
    int64_t moff;     // offset of M in Mall
    int64_t mt0;      // first mean tile of this layer (flattened over layers)
    int64_t vs0;      // first v-partial slot of this layer
};

struct FacArgs {
    FacLayer lay[NQS_MAX_LAYERS + 1];
    int L;
    int64_t n;
    double *Mall;     // [mtot] the layers' mean matrices, one after the other
    double *mpart;    // [splits][mtot] per-split sums of the mean matrices
    int64_t mtot;
    int splits;       // sample ranges of the mean sums
    double *m2part;   // [m2blocks] sums of squares of Mall per reduction block
    int m2blocks;
    double *vpart;    // [slots][n]
    int64_t slots;
    double *v;        // [n]
    double *m2;       // [1]
    float *T;         // [n][n]
    int64_t nt;       // 64-row tiles per side of T
};

constexpr int kFT = 64;    // tile side
constexpr int kFK = 32;    // staged contraction chunk of the VALU kernels

__device__ inline int fac_layer_of(const FacArgs &A, int64_t t, bool vslots)
{
    int l = 0;
    while (l + 1 < A.L && t >= (vslots ? A.lay[l + 1].vs0 : A.lay[l + 1].mt0)) ++l;
    return l;
}

// value of the augmented factor [F, 1] at (row k, column j), zero outside
__device__ inline double fac_aug(const float *F, int64_t ld, int d, int64_t n, int64_t k, int64_t j)
{
    if (k >= n || j > d) return 0.0;
    return j == d ? 1.0 : (double)F[k * ld + j];
}

// Sums of [U,1]^T [V,1] over the samples of one split (blockIdx.y), one 64 x 64
// tile of one layer per block (blockIdx.x), to mpart.
__global__ void __launch_bounds__(256) fac_mean_kernel(FacArgs A)
{
    __shared__ double Us[kFK][kFT], Vs[kFK][kFT];
    const int l = fac_layer_of(A, blockIdx.x, false);
    const FacLayer &y = A.lay[l];
    const int64_t t = blockIdx.x - y.mt0;
    const int ctiles = (y.dv + 1 + kFT - 1) / kFT;
    const int r0 = (int)(t / ctiles) * kFT, c0 = (int)(t % ctiles) * kFT;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int64_t kb = blockIdx.y * A.n / A.splits, ke = (blockIdx.y + 1) * A.n / A.splits;
    double acc[4][4] = {};
    for (int64_t k0 = kb; k0 < ke; k0 += kFK) {
        for (int e = tid; e < kFK * kFT; e += 256) {
            const int kk = e / kFT, j = e % kFT;
            const int64_t k = k0 + kk < ke ? k0 + kk : A.n;   // A.n reads as zero
            Us[kk][j] = fac_aug(y.U, y.ldu, y.du, A.n, k, r0 + j);
            Vs[kk][j] = fac_aug(y.V, y.ldv, y.dv, A.n, k, c0 + j);
        }
        __syncthreads();
        for (int kk = 0; kk < kFK; ++kk) {
            double u[4], v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) u[i] = Us[kk][ty * 4 + i];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = Vs[kk][tx * 4 + i];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(u[i], v[j], acc[i][j]);
        }
        __syncthreads();
    }
    double *out = A.mpart + (int64_t)blockIdx.y * A.mtot + y.moff;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + ty * 4 + i, c = c0 + tx * 4 + j;
            if (r <= y.du && c <= y.dv) out[(int64_t)r * (y.dv + 1) + c] = acc[i][j];
        }
}

// M_l = (1/n) (sum of the splits in order), masked: the (du, dv) corner is 0 and
// row du (the mean of V alone) is kept only when c = 1.  Per block, the sum of
// squares of its entries goes to m2part.
__global__ void __launch_bounds__(256) fac_mean_reduce_kernel(FacArgs A)
{
    __shared__ double red[256];
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double m = 0.0;
    if (e < A.mtot) {
        int l = 0;
        while (l + 1 < A.L && e >= A.lay[l + 1].moff) ++l;
        const FacLayer &y = A.lay[l];
        const int64_t q = e - y.moff;
        const int r = (int)(q / (y.dv + 1)), c = (int)(q - (int64_t)r * (y.dv + 1));
        double s = 0.0;
        for (int sp = 0; sp < A.splits; ++sp) s += A.mpart[(int64_t)sp * A.mtot + e];
        m = s / (double)A.n;
        if (r == y.du && (c == y.dv || !y.c)) m = 0.0;
        A.Mall[e] = m;
    }
    red[threadIdx.x] = m * m;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) A.m2part[blockIdx.x] = red[0];
}

// vpart[slot][k] = sum over the slot's 64 rows r of [U_k,1]_r (M [V_k,1])_r
__global__ void __launch_bounds__(256) fac_v_kernel(FacArgs A)
{
    __shared__ double Vs[kFK][kFT + 1], Ms[kFK][kFT + 1];
    const int l = fac_layer_of(A, blockIdx.y, true);
    const FacLayer &y = A.lay[l];
    const int r0 = (int)(blockIdx.y - y.vs0) * kFT;
    const int64_t k0 = (int64_t)blockIdx.x * kFT;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int ldm = y.dv + 1;
    double acc[4][4] = {};   // [sample ty*4+i][row tx*4+j]
    for (int c0 = 0; c0 <= y.dv; c0 += kFK) {
        for (int e = tid; e < kFK * kFT; e += 256) {
            const int kk = e % kFK, j = e / kFK;   // consecutive threads along the contraction
            Vs[kk][j] = fac_aug(y.V, y.ldv, y.dv, A.n, k0 + j, c0 + kk);
            const int r = r0 + j, c = c0 + kk;
            Ms[kk][j] = (r <= y.du && c <= y.dv) ? y.M[(int64_t)r * ldm + c] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < kFK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Vs[kk][ty * 4 + i];
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = Ms[kk][tx * 4 + i];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t k = k0 + ty * 4 + i;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) s = fma(fac_aug(y.U, y.ldu, y.du, A.n, k, r0 + tx * 4 + j), acc[i][j], s);
        // the 16 lanes of one sample row are consecutive: fixed-order butterfly
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 16);
        if (tx == 0 && k < A.n) A.vpart[(int64_t)blockIdx.y * A.n + k] = s;
    }
}

// v[k] = sum of the slots in order; block 0 also sums |mu|^2 from the reduction blocks
__global__ void __launch_bounds__(256) fac_vsum_kernel(FacArgs A)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < A.n) {
        double s = 0.0;
        for (int64_t q = 0; q < A.slots; ++q) s += A.vpart[q * A.n + k];
        A.v[k] = s;
    }
    if (blockIdx.x != 0) return;
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < A.m2blocks; b += blockDim.x) s += A.m2part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) A.m2[0] = red[0];
}

// Tile (bi, bj), bi <= bj, of the upper triangle in row-major order.
__device__ inline void fac_tile(int64_t t, int64_t nt, int64_t &bi, int64_t &bj)
{
    const double a = (double)(2 * nt + 1);
    int64_t r = (int64_t)((a - sqrt(a * a - 8.0 * (double)t)) * 0.5);
    r = r < 0 ? 0 : (r > nt - 1 ? nt - 1 : r);
    auto start = [nt](int64_t row) { return row * nt - row * (row - 1) / 2; };
    while (r > 0 && start(r) > t) --r;
    while (r + 1 < nt && start(r + 1) <= t) ++r;
    bi = r;
    bj = r + (t - start(r));
}

constexpr int kGK16 = 16;            // contraction step of the matrix-core kernel
constexpr int kGLd16 = kGK16 + 1;    // LDS row stride (floats)

// acc[a][b] (16 x 16 blocks of the wave's 32 x 32 quadrant) += F_I F_J^T over the first d columns
__device__ inline void fac_gram_accumulate(const float *__restrict__ F, int64_t ld, int d, int64_t n, int64_t I0,
                                           int64_t J0, float *As, float *Bs, f64x4 (&acc)[2][2])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int row = tid >> 2, k4 = (tid & 3) * 4;   // staging: 64 rows x 16 columns, 4 per thread
    const int li = lane & 15, lk = lane >> 4;
    for (int k0 = 0; k0 < d; k0 += kGK16) {
        const int64_t gi = I0 + row, gj = J0 + row;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + k4 + e;
            As[row * kGLd16 + k4 + e] = (gi < n && k < d) ? F[gi * ld + k] : 0.0f;
            Bs[row * kGLd16 + k4 + e] = (gj < n && k < d) ? F[gj * ld + k] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kGK16 / 4; ++s) {
            const int kk = s * 4 + lk;
            double av[2], bv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                av[q] = (double)As[(wm + 16 * q + li) * kGLd16 + kk];
                bv[q] = (double)Bs[(wn + 16 * q + li) * kGLd16 + kk];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) fac_gram_kernel(FacArgs A)
{
    __shared__ float As[kFT * kGLd16], Bs[kFT * kGLd16];
    // consecutive tiles (which share their row panel) on one XCD
    const int64_t tiles = A.nt * (A.nt + 1) / 2;
    const int64_t x = blockIdx.x, g = gridDim.x;
    const int64_t q8 = g >> 3, r8 = g & 7, xcd = x & 7;
    const int64_t t = xcd * q8 + min(xcd, r8) + (x >> 3);
    if (t >= tiles) return;
    int64_t bi, bj;
    fac_tile(t, A.nt, bi, bj);
    const int64_t I0 = bi * kFT, J0 = bj * kFT;

    f64x4 K[2][2], gu[2][2], gv[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) K[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < A.L; ++l) {
        const FacLayer &y = A.lay[l];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) gu[a][b] = gv[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
        fac_gram_accumulate(y.U, y.ldu, y.du, A.n, I0, J0, As, Bs, gu);
        fac_gram_accumulate(y.V, y.ldv, y.dv, A.n, I0, J0, As, Bs, gv);
        const double c = (double)y.c;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) K[a][b][r] += fma(gu[a][b][r] + c, gv[a][b][r] + 1.0, -c);
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const double inv = 1.0 / (double)A.n, m2 = A.m2[0];
    // D[i][j] of a 16 x 16 FP64 block: j = lane % 16, i = lane / 16 + 4 * register
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = I0 + wm + 16 * a + (lane >> 4) + 4 * r;
                const int64_t gj = J0 + wn + 16 * b + (lane & 15);
                if (gi >= A.n || gj >= A.n || (bi == bj && gi > gj)) continue;
                const float tv = (float)((K[a][b][r] - A.v[gi] - A.v[gj] + m2) * inv);
                A.T[gi * A.n + gj] = tv;
                if (gi != gj) A.T[gj * A.n + gi] = tv;
            }
}

__global__ void spins_to_f32_kernel(const int8_t *__restrict__ s, int64_t count, float *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) out[i] = (float)s[i];
}

// ---- host ----

// Launch geometry shared by the workspace size and the launch.
struct FacPlan {
    int64_t mt = 0, mtot = 0, vs = 0;
    int splits = 1, m2blocks = 1;
};

static FacPlan fac_plan(const FacLayerDesc *lay, int L, int64_t n)
{
    FacPlan p;
    for (int l = 0; l < L; ++l) {
        const int64_t rt = (lay[l].du + 1 + kFT - 1) / kFT, ct = (lay[l].dv + 1 + kFT - 1) / kFT;
        p.mt += rt * ct;
        p.mtot += (int64_t)(lay[l].du + 1) * (lay[l].dv + 1);
        p.vs += rt;
    }
    // enough sample splits for about eight blocks per compute unit, at least 64 samples each
    const int64_t want = ((int64_t)device_cus() * 8 + p.mt - 1) / p.mt;
    p.splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, n / 64, 1024}));
    p.m2blocks = (int)((p.mtot + 255) / 256);
    return p;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t fac_workspace_bytes(const FacLayerDesc *lay, int L, int64_t n)
{
    const FacPlan p = fac_plan(lay, L, n);
    return round256(sizeof(double) * (size_t)p.mtot) + round256(sizeof(double) * (size_t)p.splits * p.mtot) +
           round256(sizeof(double) * (size_t)p.m2blocks) + round256(sizeof(double) * (size_t)p.vs * (size_t)n) +
           round256(sizeof(double) * (size_t)n) + 256;
}

nqs_status launch_fac_gram(const FacLayerDesc *lay, int L, int64_t n, float *T, void *wsp, hipStream_t stream)
{
    if (L < 1 || L > NQS_MAX_LAYERS + 1) return set_error(NQS_EINVAL, "bad factor layer count");
    const FacPlan p = fac_plan(lay, L, n);
    FacArgs A;
    A.L = L;
    A.n = n;
    A.T = T;
    char *ws = (char *)wsp;
    A.Mall = (double *)ws;
    ws += round256(sizeof(double) * (size_t)p.mtot);
    A.mpart = (double *)ws;
    ws += round256(sizeof(double) * (size_t)p.splits * p.mtot);
    A.m2part = (double *)ws;
    ws += round256(sizeof(double) * (size_t)p.m2blocks);
    A.vpart = (double *)ws;
    ws += round256(sizeof(double) * (size_t)p.vs * (size_t)n);
    A.v = (double *)ws;
    ws += round256(sizeof(double) * (size_t)n);
    A.m2 = (double *)ws;
    A.mtot = p.mtot;
    A.splits = p.splits;
    A.m2blocks = p.m2blocks;
    A.slots = p.vs;
    int64_t mt = 0, vs = 0, moff = 0;
    for (int l = 0; l < L; ++l) {
        FacLayer &y = A.lay[l];
        y.U = lay[l].U;
        y.V = lay[l].V;
        y.ldu = lay[l].ldu;
        y.ldv = lay[l].ldv;
        y.du = lay[l].du;
        y.dv = lay[l].dv;
        y.c = lay[l].c;
        y.moff = moff;
        y.M = A.Mall + moff;
        moff += (int64_t)(y.du + 1) * (y.dv + 1);
        y.mt0 = mt;
        mt += (int64_t)((y.du + 1 + kFT - 1) / kFT) * ((y.dv + 1 + kFT - 1) / kFT);
        y.vs0 = vs;
        vs += (y.du + 1 + kFT - 1) / kFT;
    }
    A.nt = (n + kFT - 1) / kFT;
    const int64_t tiles = A.nt * (A.nt + 1) / 2;
    const int64_t ktiles = (n + kFT - 1) / kFT;
    if (tiles > INT32_MAX || mt > INT32_MAX || ktiles > INT32_MAX || vs > 65535 || p.m2blocks > INT32_MAX / 2)
        return set_error(NQS_EINVAL, "sample-space Gram matrix too large");

    hipLaunchKernelGGL(fac_mean_kernel, dim3((unsigned)mt, (unsigned)p.splits), dim3(256), 0, stream, A);
    hipLaunchKernelGGL(fac_mean_reduce_kernel, dim3((unsigned)p.m2blocks), dim3(256), 0, stream, A);
    hipLaunchKernelGGL(fac_v_kernel, dim3((unsigned)ktiles, (unsigned)vs), dim3(256), 0, stream, A);
    hipLaunchKernelGGL(fac_vsum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, A);
    hipLaunchKernelGGL(fac_gram_kernel, dim3((unsigned)tiles), dim3(256), 0, stream, A);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

void launch_spins_to_f32(const int8_t *s, int64_t count, float *out, hipStream_t stream)
{
    hipLaunchKernelGGL(spins_to_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, s, count,
                       out);
}

}  // namespace nqs
