// Stochastic reconfiguration step in sample space (App. I.2, Eq. eq:smat, with
// the forces of Eq. eq:forces).  The update direction delta solves
//     (S + shift) delta = F,   S = Obar^T Obar / n,   F = Obar^T e / n,
// e = eps - mean(eps).  S and T = Obar Obar^T / n share their non-zero
// spectrum, and (S + shift)^{-1} Obar^T = Obar^T (T + shift)^{-1}, so
//     delta = Obar^T y / n,   (T + shift) y = e:
// an n x n system in place of a P x P one.  Obar^T y = O^T (y - mean y), one
// vector-Jacobian product of the log-derivatives.
//
// nqs_sr_solve: Jacobi-preconditioned conjugate gradients, FP64 vectors and
//   scalars, FP32 T read once per iteration (four rows per wave, FP64 sums).
//   Up to n = 65536 an iteration is two launches: the product with its
//   per-row p.Ap, then one block for the scalars and the vector updates.
//   Every reduction is a fixed-order single-block tree, so the iterates do
//   not depend on timing.  Scalars stay on the device (one slot per
//   iteration); the host reads the residual every kCheck iterations.
// nqs_sr_update: delta = O^T (y - mean y) / n through the FP32 copy's VJP,
//   master -= lr * delta in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "internal.h"
#include "nqs.h"

namespace nqs {

constexpr int kSumThreads = 1024;
constexpr int kCheck = 8;
constexpr int64_t kFusedMax = 65536;   // the one-block iteration of the Jacobi CG up to this n

// out[0] = sum_k a[k] * (b ? b[k] : 1), one block, fixed order
__global__ void __launch_bounds__(kSumThreads) sr_dot_kernel(const double *__restrict__ a,
                                                             const double *__restrict__ b, int64_t n,
                                                             double *__restrict__ out)
{
    __shared__ double red[kSumThreads];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += kSumThreads) s = fma(a[k], b ? b[k] : 1.0, s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kSumThreads / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Ap = (T + shift) p, one wave per row, T with leading dimension ld; over
// columns k < n (mode 0), k <= row (1: lower triangle) or k >= row (2: upper).
// With vec (rows of T and p 16-byte aligned) the columns from the first
// multiple of four on are read four at a time.
__global__ void __launch_bounds__(256) sr_matvec_kernel(const float *__restrict__ T, int64_t ld,
                                                        const double *__restrict__ p, int64_t n, double shift,
                                                        int mode, int vec, double *__restrict__ Ap)
{
    const int64_t row = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float *t = T + row * ld;
    const int64_t lo = mode == 2 ? row : 0, hi = mode == 1 ? row + 1 : n;
    double s = 0.0;
    int64_t k0 = lo;
    if (vec) {
        const int64_t a = std::min<int64_t>(hi, (lo + 3) & ~(int64_t)3);
        if (lo + lane < a) s = fma((double)t[lo + lane], p[lo + lane], s);
        const int64_t n4 = (hi - a) >> 2;
        for (int64_t q = lane; q < n4; q += 64) {
            const int64_t c = a + 4 * q;
            const float4 v = *(const float4 *)(t + c);
            const double2 pa = *(const double2 *)(p + c), pb = *(const double2 *)(p + c + 2);
            s = fma((double)v.x, pa.x, s);
            s = fma((double)v.y, pa.y, s);
            s = fma((double)v.z, pb.x, s);
            s = fma((double)v.w, pb.y, s);
        }
        k0 = a + (n4 << 2);
    }
    for (int64_t k = k0 + lane; k < hi; k += 64) s = fma((double)t[k], p[k], s);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) Ap[row] = s + shift * p[row];
}

// Ap = (T + shift) p over all n columns, four consecutive rows per wave (T's
// row count is n, leading dimension ld); pr[row] = p[row] Ap[row] when pr is
// given.  Each lane reads T four floats at a time from every row and p once
// per column group for all four rows, when vec says T's rows and p are 16-byte
// aligned; otherwise element by element.  Rows past n read row n - 1 and store
// nothing.
constexpr int kRowsPerWave = 4;

__global__ void __launch_bounds__(256) sr_matvec_rows_kernel(const float *__restrict__ T, int64_t ld,
                                                             const double *__restrict__ p, int64_t n, double shift,
                                                             int vec, double *__restrict__ Ap, double *__restrict__ pr)
{
    constexpr int R = kRowsPerWave;
    const int64_t row0 = (blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6)) * R;
    const int lane = threadIdx.x & 63;
    if (row0 >= n) return;
    const float *t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = T + std::min<int64_t>(row0 + r, n - 1) * ld;
    double s[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = 0.0;
    int64_t k0 = 0;
    if (vec) {
        const int64_t n4 = n >> 2;
#pragma unroll 2
        for (int64_t q = lane; q < n4; q += 64) {
            const double2 pa = *(const double2 *)(p + 4 * q), pb = *(const double2 *)(p + 4 * q + 2);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float4 v = *(const float4 *)(t[r] + 4 * q);
                s[r] = fma((double)v.x, pa.x, s[r]);
                s[r] = fma((double)v.y, pa.y, s[r]);
                s[r] = fma((double)v.z, pb.x, s[r]);
                s[r] = fma((double)v.w, pb.y, s[r]);
            }
        }
        k0 = n4 << 2;
    }
    for (int64_t k = k0 + lane; k < n; k += 64) {
        const double pk = p[k];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = fma((double)t[r][k], pk, s[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s[r] += __shfl_xor(s[r], o, 64);
    }
    if (lane < R && row0 + lane < n) {
        double sl = s[0];
#pragma unroll
        for (int r = 1; r < R; ++r) sl = lane == r ? s[r] : sl;
        const int64_t row = row0 + lane;
        const double a = sl + shift * p[row];
        Ap[row] = a;
        if (pr) pr[row] = p[row] * a;
    }
}

// grid of sr_matvec_rows_kernel for n rows, and whether its vector loads apply
inline unsigned sr_rows_blocks(int64_t n) { return (unsigned)((n + 4 * kRowsPerWave - 1) / (4 * kRowsPerWave)); }
inline int sr_rows_vec(const float *T, int64_t ld, const double *p)
{
    return ((uintptr_t)T % 16 == 0 && ld % 4 == 0 && (uintptr_t)p % 16 == 0) ? 1 : 0;
}

// fixed-order sum of v[0..n) by one block of kSumThreads (every thread returns the total)
__device__ inline double sr_block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kSumThreads / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// The rest of Jacobi-preconditioned CG iteration k in one block: pAp from the
// per-row products, alpha, x += alpha p, r -= alpha Ap, z = r d, rz[k + 1] =
// r.z, rr[k] = r.r, beta, p = z + beta p.
__global__ void __launch_bounds__(kSumThreads) sr_iter_kernel(const double *__restrict__ pr, const double *__restrict__ Ap,
                                                              const double *__restrict__ d, int64_t n, int k,
                                                              double *__restrict__ rz, double *__restrict__ rr,
                                                              double *__restrict__ x, double *__restrict__ r,
                                                              double *__restrict__ z, double *__restrict__ p)
{
    __shared__ double red[kSumThreads];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kSumThreads) a += pr[i];
    const double pap = sr_block_sum(a, red);
    const double alpha = pap != 0.0 ? rz[k] / pap : 0.0;
    double zr = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kSumThreads) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, Ap[i], r[i]);
        const double zi = ri * d[i];
        r[i] = ri;
        z[i] = zi;
        zr = fma(ri, zi, zr);
        q = fma(ri, ri, q);
    }
    const double rz1 = sr_block_sum(zr, red);
    const double rr1 = sr_block_sum(q, red);
    const double beta = rz[k] != 0.0 ? rz1 / rz[k] : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kSumThreads) p[i] = fma(beta, p[i], z[i]);
    if (threadIdx.x == 0) {
        rz[k + 1] = rz1;
        rr[k] = rr1;
    }
}

// b = eps - mean (sum[0] = sum of eps); x = 0, r = b; with d: d = 1 / (diag(T) + shift), z = r d, p = z
__global__ void sr_init_kernel(const float *__restrict__ T, const double *__restrict__ eps,
                               const double *__restrict__ sum, int64_t n, double shift, double *__restrict__ d,
                               double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
                               double *__restrict__ p)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double b = eps[k] - sum[0] / (double)n;
    x[k] = 0.0;
    r[k] = b;
    if (!d) return;   // z and p are set by the caller's preconditioner
    const double dk = (double)T[k * n + k] + shift;
    const double inv = dk > 0.0 ? 1.0 / dk : 1.0;
    d[k] = inv;
    z[k] = b * inv;
    p[k] = b * inv;
}

// alpha = rz / pAp;  x += alpha p;  r -= alpha Ap;  with d: z = r d
__global__ void sr_step_kernel(const double *__restrict__ rz, const double *__restrict__ pap, int64_t n,
                               const double *__restrict__ d, const double *__restrict__ p,
                               const double *__restrict__ Ap, double *__restrict__ x, double *__restrict__ r,
                               double *__restrict__ z)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double alpha = pap[0] != 0.0 ? rz[0] / pap[0] : 0.0;
    x[k] = fma(alpha, p[k], x[k]);
    const double rk = fma(-alpha, Ap[k], r[k]);
    r[k] = rk;
    if (d) z[k] = rk * d[k];
}

// p = z + (rz_new / rz_old) p
__global__ void sr_dir_kernel(const double *__restrict__ rz_old, const double *__restrict__ rz_new, int64_t n,
                              const double *__restrict__ z, double *__restrict__ p)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double beta = rz_old[0] != 0.0 ? rz_new[0] / rz_old[0] : 0.0;
    p[k] = fma(beta, p[k], z[k]);
}

// yc = (y - mean y) / n as FP32 (sum[0] = sum of y)
__global__ void sr_center_kernel(const double *__restrict__ y, const double *__restrict__ sum, int64_t n,
                                 float *__restrict__ yc)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) yc[k] = (float)((y[k] - sum[0] / (double)n) / (double)n);
}

__global__ void sr_apply_kernel(const float *__restrict__ g, int64_t P, double lr, double *__restrict__ master)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < P) master[p] = fma(-lr, (double)g[p], master[p]);
}

static inline size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace nqs

using namespace nqs;

extern "C" {

nqs_status nqs_sr_solve(const float *T, const double *eloc, int64_t n, double shift, double tol, int32_t max_iter,
                        double *y, int32_t *iters, double *rel_resid, void *stream)
{
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!T || !eloc || !y) return set_error(NQS_EINVAL, "NULL T/eloc/y");
    if (!(shift >= 0.0) || !(tol > 0.0) || max_iter < 1) return set_error(NQS_EINVAL, "need shift >= 0, tol > 0, max_iter >= 1");
    if (n > (int64_t)INT32_MAX * 4) return set_error(NQS_EINVAL, "n too large");
    hipStream_t s = (hipStream_t)stream;
    const size_t vec = r256(sizeof(double) * (size_t)n);
    const size_t nsc = (size_t)max_iter + 2;
    char *ws = (char *)workspace_slot(1, 6 * vec + 3 * r256(sizeof(double) * nsc) + 256, s);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    double *d = (double *)ws, *r = (double *)(ws + vec), *z = (double *)(ws + 2 * vec), *p = (double *)(ws + 3 * vec),
           *Ap = (double *)(ws + 4 * vec), *prow = (double *)(ws + 5 * vec);
    double *rz = (double *)(ws + 6 * vec);                       // rz[k]: r.z after k iterations
    double *pap = rz + r256(sizeof(double) * nsc) / sizeof(double);     // p.Ap, or r.r in the fused path
    double *misc = pap + r256(sizeof(double) * nsc) / sizeof(double);   // [0] sum of eps, [1] b.b, [2] r.r
    double *rrs = pap;
    const unsigned eb = (unsigned)((n + 255) / 256);
    const unsigned rb = sr_rows_blocks(n);
    const int rv = sr_rows_vec(T, n, p);

    hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, eloc, (const double *)nullptr, n, misc);
    hipLaunchKernelGGL(sr_init_kernel, dim3(eb), dim3(256), 0, s, T, eloc, misc, n, shift, d, y, r, z, p);
    hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, r, n, misc + 1);
    hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, z, n, rz);
    NQS_HIP_TRY(hipGetLastError());
    double bb = 0.0;
    NQS_HIP_TRY(hipMemcpyAsync(&bb, misc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    NQS_HIP_TRY(hipStreamSynchronize(s));
    double rel = 0.0;
    int k = 0;
    if (bb > 0.0 && n <= kFusedMax) {
        // two launches per iteration: the matrix-vector product with its per-row p.Ap, then one block for
        // the rest; r.r of every iteration is kept, the host reads it every kCheck iterations
        rel = 1.0;
        while (k < max_iter) {
            hipLaunchKernelGGL(sr_matvec_rows_kernel, dim3(rb), dim3(256), 0, s, T, n, (const double *)p, n, shift,
                               rv, Ap, prow);
            hipLaunchKernelGGL(sr_iter_kernel, dim3(1), dim3(kSumThreads), 0, s, prow, Ap, d, n, k, rz, rrs, y, r, z, p);
            ++k;
            if (k % kCheck == 0 || k == max_iter) {
                NQS_HIP_TRY(hipGetLastError());
                double rr = 0.0;
                NQS_HIP_TRY(hipMemcpyAsync(&rr, rrs + (k - 1), sizeof(double), hipMemcpyDeviceToHost, s));
                NQS_HIP_TRY(hipStreamSynchronize(s));
                rel = std::sqrt(rr / bb);
                if (!(rel > tol)) break;   // converged (or NaN: stop and report it)
            }
        }
    } else if (bb > 0.0) {
        rel = 1.0;
        while (k < max_iter) {
            hipLaunchKernelGGL(sr_matvec_rows_kernel, dim3(rb), dim3(256), 0, s, T, n, (const double *)p, n, shift,
                               rv, Ap, (double *)nullptr);
            hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, p, Ap, n, pap + k);
            hipLaunchKernelGGL(sr_step_kernel, dim3(eb), dim3(256), 0, s, rz + k, pap + k, n, d, p, Ap, y, r, z);
            hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, z, n, rz + k + 1);
            hipLaunchKernelGGL(sr_dir_kernel, dim3(eb), dim3(256), 0, s, rz + k, rz + k + 1, n, z, p);
            ++k;
            if (k % kCheck == 0 || k == max_iter) {
                hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, r, n, misc + 2);
                NQS_HIP_TRY(hipGetLastError());
                double rr = 0.0;
                NQS_HIP_TRY(hipMemcpyAsync(&rr, misc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
                NQS_HIP_TRY(hipStreamSynchronize(s));
                rel = std::sqrt(rr / bb);
                if (!(rel > tol)) break;   // converged (or NaN: stop and report it)
            }
        }
    }
    if (iters) *iters = k;
    if (rel_resid) *rel_resid = rel;
    return NQS_OK;
}

nqs_status nqs_sr_solve_mixed(const float *T, const double *eloc, int64_t n, double shift, int32_t factor_dtype,
                              double tol, int32_t max_iter, double *y, int32_t *iters, double *rel_resid,
                              int64_t *n_pivots_fixed, int32_t *factor_used, void *stream)
{
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (n > 65536) return set_error(NQS_EINVAL, "n must be at most 65536 (two n x n FP32 factors are formed)");
    if (!T || !eloc || !y) return set_error(NQS_EINVAL, "NULL T/eloc/y");
    if (!(shift >= 0.0) || !(tol > 0.0) || max_iter < 1) return set_error(NQS_EINVAL, "need shift >= 0, tol > 0, max_iter >= 1");
    if (factor_dtype != NQS_F32 && factor_dtype != NQS_BF16 && factor_dtype != NQS_F16)
        return set_error(NQS_EINVAL, "factor dtype must be F32, BF16 or F16");
    hipStream_t s = (hipStream_t)stream;
    const size_t fac = r256(mix_workspace_bytes(n));
    const size_t vec = r256(sizeof(double) * (size_t)n);
    const size_t nsc = (size_t)max_iter + 2;
    char *ws = (char *)workspace_slot(1, fac + 6 * vec + 3 * r256(sizeof(double) * nsc) + 256, s);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    char *v = ws + fac;
    double *r = (double *)v, *z = (double *)(v + vec), *p = (double *)(v + 2 * vec), *Ap = (double *)(v + 3 * vec),
           *u = (double *)(v + 4 * vec), *d = (double *)(v + 5 * vec);
    double *rz = (double *)(v + 6 * vec);
    double *pap = rz + r256(sizeof(double) * nsc) / sizeof(double);
    double *misc = pap + r256(sizeof(double) * nsc) / sizeof(double);   // [0] sum of eps, [1] b.b, [2] r.r, [3] pivots
    unsigned long long *nfix = (unsigned long long *)(misc + 3);
    const unsigned eb = (unsigned)((n + 255) / 256), mb = (unsigned)((n + 3) / 4);
    const unsigned rb = sr_rows_blocks(n);
    const int rv = sr_rows_vec(T, n, p);

    // Attempts: the requested format, then an FP32 factor, then the Jacobi
    // preconditioner (-1).  A reduced-precision factor that had to replace
    // more than n / 8 pivots (T + shift is too ill-conditioned for the
    // format) is not used; an attempt whose preconditioned residual is not a
    // positive finite number, or whose iteration turns non-finite, is
    // abandoned for the next one.
    int fmts[3] = {factor_dtype, NQS_F32, -1};
    const int nf = factor_dtype == NQS_F32 ? 2 : 3;
    if (factor_dtype == NQS_F32) fmts[1] = -1;
    double rel = 0.0;
    int k = 0;
    unsigned long long fixed_total = 0;
    int used = -1;
    for (int att = 0; att < nf; ++att) {
        const int fmt = fmts[att];
        float *Lin = nullptr, *LinT = nullptr;
        int64_t np = 0;
        if (fmt >= 0) {
            nqs_status st = launch_zero_u64(nfix, 1, s);
            if (st != NQS_OK) return st;
            st = mix_factor(T, n, shift, fmt, ws, &Lin, &LinT, &np, nfix, s);
            if (st != NQS_OK) return st;
            unsigned long long fixed = 0;
            NQS_HIP_TRY(hipMemcpyAsync(&fixed, nfix, sizeof(fixed), hipMemcpyDeviceToHost, s));
            NQS_HIP_TRY(hipStreamSynchronize(s));
            fixed_total = fixed;
            if (fmt != NQS_F32 && fixed > (unsigned long long)(n / 8)) continue;
        }
        // z = M^{-1} r: L^{-T} (L^{-1} r), or r / diag with the Jacobi preconditioner
        auto precond = [&]() {
            hipLaunchKernelGGL(sr_matvec_kernel, dim3(mb), dim3(256), 0, s, (const float *)Lin, np,
                               (const double *)r, n, 0.0, 1, sr_rows_vec(Lin, np, r), u);
            hipLaunchKernelGGL(sr_matvec_kernel, dim3(mb), dim3(256), 0, s, (const float *)LinT, np,
                               (const double *)u, n, 0.0, 2, sr_rows_vec(LinT, np, u), z);
        };
        double *dj = fmt >= 0 ? nullptr : d;
        hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, eloc, (const double *)nullptr, n, misc);
        hipLaunchKernelGGL(sr_init_kernel, dim3(eb), dim3(256), 0, s, T, eloc, misc, n, shift, dj, y, r, z, p);
        hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, r, n, misc + 1);
        if (fmt >= 0) {
            precond();
            NQS_HIP_TRY(hipMemcpyAsync(p, z, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        }
        hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, z, n, rz);
        NQS_HIP_TRY(hipGetLastError());
        double bb = 0.0, rz0 = 0.0;
        NQS_HIP_TRY(hipMemcpyAsync(&bb, misc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        NQS_HIP_TRY(hipMemcpyAsync(&rz0, rz, sizeof(double), hipMemcpyDeviceToHost, s));
        NQS_HIP_TRY(hipStreamSynchronize(s));
        rel = 0.0;
        k = 0;
        used = fmt;
        if (!(bb > 0.0)) break;
        if (!(rz0 > 0.0) || !std::isfinite(rz0)) continue;   // preconditioner unusable
        rel = 1.0;
        while (k < max_iter) {
            hipLaunchKernelGGL(sr_matvec_rows_kernel, dim3(rb), dim3(256), 0, s, T, n, (const double *)p, n, shift,
                               rv, Ap, (double *)nullptr);
            hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, p, Ap, n, pap + k);
            hipLaunchKernelGGL(sr_step_kernel, dim3(eb), dim3(256), 0, s, rz + k, pap + k, n, (const double *)dj, p,
                               Ap, y, r, z);
            if (fmt >= 0) precond();
            hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, z, n, rz + k + 1);
            hipLaunchKernelGGL(sr_dir_kernel, dim3(eb), dim3(256), 0, s, rz + k, rz + k + 1, n, z, p);
            ++k;
            // a good factor converges in a few iterations: check every iteration
            if (fmt >= 0 || k % kCheck == 0 || k == max_iter) {
                hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, r, r, n, misc + 2);
                NQS_HIP_TRY(hipGetLastError());
                double rr = 0.0;
                NQS_HIP_TRY(hipMemcpyAsync(&rr, misc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
                NQS_HIP_TRY(hipStreamSynchronize(s));
                rel = std::sqrt(rr / bb);
                if (!(rel > tol)) break;   // converged, or NaN
            }
        }
        if (std::isfinite(rel)) break;
    }
    if (iters) *iters = k;
    if (rel_resid) *rel_resid = rel;
    if (n_pivots_fixed) *n_pivots_fixed = (int64_t)fixed_total;
    if (factor_used) *factor_used = used;
    return NQS_OK;
}

nqs_status nqs_sr_solve_complex(const float *T2, const double *eloc_re, const double *eloc_im, int64_t n, double shift,
                                double tol, int32_t max_iter, double *y2, int32_t *iters, double *rel_resid, void *stream)
{
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!T2 || !eloc_re || !eloc_im || !y2) return set_error(NQS_EINVAL, "NULL T2/eloc/y2");
    if (!(shift >= 0.0) || !(tol > 0.0) || max_iter < 1) return set_error(NQS_EINVAL, "need shift >= 0, tol > 0, max_iter >= 1");
    if (n > (int64_t)INT32_MAX) return set_error(NQS_EINVAL, "n too large");
    double *e2 = nullptr;
    nqs_status st = cplx_sr_rhs(eloc_re, eloc_im, n, &e2, (hipStream_t)stream);
    if (st != NQS_OK) return st;
    // both halves are centred, so the solver's own centring (by the mean of all 2n values) changes nothing
    return nqs_sr_solve(T2, e2, 2 * n, shift, tol, max_iter, y2, iters, rel_resid, stream);
}

nqs_status nqs_sr_update(nqs_model *m, const int8_t *samples, int64_t n, const double *y, double lr, double *master,
                         void *stream)
{
    if (!m) return set_error(NQS_EINVAL, "NULL model");
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!samples || !y || !master) return set_error(NQS_EINVAL, "NULL samples/y/master");
    hipStream_t s = (hipStream_t)stream;
    if (m->desc.arch == NQS_CRBM) return crbm_sr_update(m, samples, n, y, lr, master, s);   // y holds 2n values
    const int64_t P = m->P;
    const size_t yb = r256(sizeof(float) * (size_t)n), gb = r256(sizeof(float) * (size_t)P);
    char *ws = (char *)workspace_slot(1, yb + gb + 256, s);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    float *yc = (float *)ws, *g = (float *)(ws + yb);
    double *sum = (double *)(ws + yb + gb);
    hipLaunchKernelGGL(sr_dot_kernel, dim3(1), dim3(kSumThreads), 0, s, y, (const double *)nullptr, n, sum);
    hipLaunchKernelGGL(sr_center_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, sum, n, yc);
    NQS_HIP_TRY(hipGetLastError());
    nqs_status st = m->desc.arch == NQS_RBM      ? rbm_logpsi_grad(m, samples, n, nullptr, nullptr, yc, g, s, 0, P)
                    : m->desc.arch == NQS_RESCNN ? cnn_logpsi_grad(m, samples, n, nullptr, nullptr, yc, g, s)
                                                 : ffnn_logpsi_grad(m, samples, n, nullptr, nullptr, yc, g, s, 0, P);
    if (st != NQS_OK) return st;
    hipLaunchKernelGGL(sr_apply_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, g, P, lr, master);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // extern "C"
