// Complex-parameter RBM: log psi = sum_i a_i s_i + sum_j log cosh(theta_j),
// theta = W s + b, a, b, W complex; the sampled distribution is |psi|^2 =
// exp(2 Re log psi).  Flipping site i multiplies psi by
//     exp(-2 a_i s_i) prod_j (C_ji - s_i t_j S_ji),
// C = cosh 2W, S = sinh 2W, t = tanh theta (all complex).
//
// Sampler: one chain per group of lanes, lanes over hidden units, complex
// (cosh theta, sinh theta) carried through accepted flips by the addition
// formulas and recomputed from W s + b every sweep (details at the kernel).
// Local energies: one sample per workgroup, one thread per site, the complex
// flip ratios summed in FP64 (real and imaginary parts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "crbm_math.h"
#include "internal.h"

namespace nqs {

constexpr int kCrbmThreads = 256;

// ---- copy ----

__global__ void crbm_build_kernel(const double *__restrict__ master, int N, int M, int dtype, CrbmDev d)
{
    const int64_t P = N + M + (int64_t)M * N;
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < N) {
        d.a[q] = make_float2((float)round_to_dtype(master[q], dtype), (float)round_to_dtype(master[P + q], dtype));
        d.a2[q] = (float)(4.0 * round_to_dtype(master[q], dtype) / 0.69314718055994531);
    } else if (q < N + M) {
        d.b[q - N] = make_float2((float)round_to_dtype(master[q], dtype), (float)round_to_dtype(master[P + q], dtype));
    } else if (q < P) {
        const int64_t r = q - N - M;
        const int j = (int)(r / N), i = (int)(r - (int64_t)j * N);
        const double wr = round_to_dtype(master[q], dtype), wi = round_to_dtype(master[P + q], dtype);
        d.Wt[(int64_t)i * M + j] = make_float2((float)wr, (float)wi);
        // cosh 2w = cosh 2x cos 2y + i sinh 2x sin 2y; sinh 2w = sinh 2x cos 2y + i cosh 2x sin 2y
        const double ch = cosh(2.0 * wr), sh = sinh(2.0 * wr), c = cos(2.0 * wi), s = sin(2.0 * wi);
        const float4 cs = make_float4((float)(ch * c), (float)(sh * s), (float)(sh * c), (float)(ch * s));
        d.CS[(int64_t)i * M + j] = cs;
        d.CSt[(int64_t)j * N + i] = cs;
    } else if (q == P) {
        d.CS[(int64_t)N * M] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);   // neutral entry for lanes past the last unit
    }
}

nqs_status crbm_build_copy(nqs_model *m, int dtype, hipStream_t stream)
{
    if (dtype == NQS_FP8_E4M3) return set_error(NQS_EUNSUPPORTED, "no FP8 copy of the complex RBM");
    const int N = m->desc.n_visible, M = m->desc.widths[0];
    Copy &c = m->copies[dtype];
    CrbmDev &d = c.crbm;
    d.N = N;
    d.M = M;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nm = (size_t)N * M;
    const size_t bytes = al(sizeof(float2) * N) + al(sizeof(float) * N) + al(sizeof(float2) * M) +
                         al(sizeof(float2) * nm) + al(sizeof(float4) * (nm + 1)) + al(sizeof(float4) * nm);
    if (!c.block) NQS_HIP_TRY(hipMalloc(&c.block, bytes));
    char *p = (char *)c.block;
    d.a = (float2 *)p;
    p += al(sizeof(float2) * N);
    d.a2 = (float *)p;
    p += al(sizeof(float) * N);
    d.b = (float2 *)p;
    p += al(sizeof(float2) * M);
    d.Wt = (float2 *)p;
    p += al(sizeof(float2) * nm);
    d.CS = (float4 *)p;
    p += al(sizeof(float4) * (nm + 1));
    d.CSt = (float4 *)p;
    const int64_t P = N + M + (int64_t)nm;
    hipLaunchKernelGGL(crbm_build_kernel, dim3((unsigned)((P + 1 + 255) / 256)), dim3(256), 0, stream, m->master, N,
                       M, dtype, d);
    NQS_HIP_TRY(hipGetLastError());
    c.valid = true;
    return NQS_OK;
}

// ---- sampler ----
//
// One chain per group of G lanes (G = 16, 32 or 64); lane g of the group owns
// hidden units j = g + qG, q < K, and spin word g (32 spins per word).  Per
// unit the chain keeps complex (c_j, s_j) proportional to (cosh theta_j,
// sinh theta_j), with c = 1 after each refresh, and per lane the running
// log2 of prod_q |c_q|^2.  With C = cosh 2W_ji and S = sinh 2W_ji, flipping
// site i gives
//   n_j = c_j C - s_i s_j S = c_j cosh(theta_j - 2 s_i W_ji) / cosh theta_j,
//   log2 |psi(s')/psi(s)|^2 = -4 Re(a_i) s_i / ln 2 + sum_j [log2 |n_j|^2 - log2 |c_j|^2],
// and an accepted flip sets c_j <- n_j, s_j <- s_j C - s_i c_j S.  The move is
// accepted iff log2 u < that log-ratio.  The squared moduli of a lane are
// multiplied (renormalised every four factors) and take one logarithm.  The
// (C, S) column of the next proposal is loaded while the current one is
// decided; the table sits in LDS when it fits, else it is read through L2.

struct CrbmSampleArgs {
    CrbmDev net;
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

constexpr int kCrbmMaxK = 8;

// theta = W s + b from the spin words; c = 1, s = tanh theta.  Returns
// Re log psi (FP32) when want_f (uniform across the group), else 0.
template <int G, int K>
__device__ __forceinline__ float crbm_refresh(const CrbmDev &net, uint32_t word, int gl, float2 (&c)[K],
                                              float2 (&sh)[K], bool want_f)
{
    const int N = net.N, M = net.M;
    constexpr int CH = K >= 6 ? 2 : 4;   // sites whose W rows are in flight together
    float2 th[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = gl + k * G;
        th[k] = j < M ? net.b[j] : make_float2(0.0f, 0.0f);
    }
    const int jl = gl + (K - 1) * G;
    const int jlast = jl < M ? jl : M - 1;          // clamp the tail slot to a valid column
    const float wlast = jl < M ? 1.0f : 0.0f;
    float as = 0.0f;
    const int NW = (N + 31) >> 5;
    for (int w = 0; w < NW; ++w) {
        const uint32_t bits = group_bcast<G>(word, w);
        const int i0 = w << 5;
        const int nb = min(32, N - i0);
        int bb = 0;
        for (; bb + CH <= nb; bb += CH) {
            float2 wv[CH][K];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const float2 *wrow = net.Wt + (size_t)(i0 + bb + q) * M;
#pragma unroll
                for (int k = 0; k < K - 1; ++k) wv[q][k] = wrow[gl + k * G];
                wv[q][K - 1] = wrow[jlast];
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const float s = ((bits >> (bb + q)) & 1u) ? 1.0f : -1.0f;
                as = fmaf(net.a[i0 + bb + q].x, s, as);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float sw = k == K - 1 ? s * wlast : s;
                    th[k].x = fmaf(wv[q][k].x, sw, th[k].x);
                    th[k].y = fmaf(wv[q][k].y, sw, th[k].y);
                }
            }
        }
        for (; bb < nb; ++bb) {
            const float2 *wrow = net.Wt + (size_t)(i0 + bb) * M;
            const float s = ((bits >> bb) & 1u) ? 1.0f : -1.0f;
            as = fmaf(net.a[i0 + bb].x, s, as);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float2 wk = wrow[k == K - 1 ? jlast : gl + k * G];
                const float sw = k == K - 1 ? s * wlast : s;
                th[k].x = fmaf(wk.x, sw, th[k].x);
                th[k].y = fmaf(wk.y, sw, th[k].y);
            }
        }
    }
    float lc = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        c[k] = make_float2(1.0f, 0.0f);
        sh[k] = ctanh(th[k]);
        if (want_f && (k < K - 1 || jl < M)) lc += clogcosh_re(th[k]);
    }
    return want_f ? as + group_sum_uniform<G>(lc) : 0.0f;
}

// Proposal (batch start + g) for lane g of a group: site, u bits, log2 u and
// the visible-bias term 4 Re(a_i) / ln 2.
struct CrbmProp {
    uint32_t i, ub;
    float l2u, a2;
};

__device__ __forceinline__ CrbmProp crbm_prop(const CrbmDev &net, uint64_t step, uint32_t gid, uint32_t inst,
                                              uint32_t key0, uint32_t key1)
{
    const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, inst << 8, key0, key1);
    CrbmProp pb;
    pb.i = (uint32_t)index_from_word(rb.r0, net.N);
    pb.ub = rb.r2 >> 8;
    pb.l2u = __builtin_amdgcn_logf((float)pb.ub * 5.9604644775390625e-8f);   // log2 u, u = ub 2^-24
    pb.a2 = net.a2[pb.i];
    return pb;
}

template <int G, int K>
__device__ __forceinline__ void crbm_column(const float4 *__restrict__ tab, int i, int M, int gl, int last_off,
                                            bool last_ok, float4 (&cs)[K])
{
    const int base = i * M + gl;
#pragma unroll
    for (int k = 0; k < K - 1; ++k) cs[k] = tab[base + k * G];
    cs[K - 1] = tab[last_ok ? base + (K - 1) * G : last_off];
}

template <int G, int K, bool LDS_TAB>
__global__ void __launch_bounds__(G == 16 ? 256 : 512) crbm_sample_kernel(CrbmSampleArgs A)
{
    extern __shared__ float4 s_ctab[];
    const int N = A.net.N, M = A.net.M;
    if constexpr (LDS_TAB) {
        const int tot = N * M + 1;   // includes the neutral entry
        for (int k = threadIdx.x; k < tot; k += blockDim.x) s_ctab[k] = A.net.CS[k];
        __syncthreads();
    }
    const int cpb = blockDim.x / G;
    const int gl = threadIdx.x % G;
    const int64_t c = (int64_t)blockIdx.x * cpb + threadIdx.x / G;
    if (c >= A.n_chains) return;   // whole groups leave together; no barrier follows

    const uint32_t gid = A.chain_id_offset + (uint32_t)c;
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    const int NW = (N + 31) >> 5;
    const int last_off = N * M;
    const bool last_ok = gl + (K - 1) * G < M;

    uint32_t word = 0;
    if (gl < NW) {
        const int nb = min(32, N - gl * 32);
        const int8_t *src = A.chain_state + (size_t)c * N + gl * 32;
        for (int bb = 0; bb < nb; ++bb) word |= (src[bb] > 0 ? 1u : 0u) << bb;
    }
    float2 cc[K], sh[K];
    crbm_refresh<G, K>(A.net, word, gl, cc, sh, false);
    float lpart = 0.0f;

    const int sw = A.sweep_size;
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * sw;
    const bool traced = c < A.n_traced;
    unsigned long long acc = 0;
    int in_sweep = 0;
    int64_t sweep = 0;

    // proposal pipeline: `cur` covers steps [base, base+G), `nxt` the next G
    uint64_t base = A.step_offset;
    CrbmProp cur = crbm_prop(A.net, base + gl, gid, A.inst, key0, key1);
    CrbmProp nxt = crbm_prop(A.net, base + G + gl, gid, A.inst, key0, key1);
    int p = 0;
    int i_c = (int)group_bcast<G>(cur.i, 0);
    uint32_t ub_c = group_bcast<G>(cur.ub, 0);
    float l2u_c = __uint_as_float(group_bcast<G>(__float_as_uint(cur.l2u), 0));
    float a2_c = __uint_as_float(group_bcast<G>(__float_as_uint(cur.a2), 0));
    float4 csA[K], csB[K];
    if constexpr (LDS_TAB) crbm_column<G, K>(s_ctab, i_c, M, gl, last_off, last_ok, csA);
    else crbm_column<G, K>(A.net.CS, i_c, M, gl, last_off, last_ok, csA);

    // one proposal: evaluate with cs_c (column of i_c), prefetch the next column into cs_n
    auto step = [&](int64_t k, float4 (&cs_c)[K], float4 (&cs_n)[K]) {
        const int pn = p + 1;
        const CrbmProp &src = pn < G ? cur : nxt;
        const int pl = pn < G ? pn : 0;
        const int i_n = (int)group_bcast<G>(src.i, pl);
        const uint32_t ub_n = group_bcast<G>(src.ub, pl);
        const float l2u_n = __uint_as_float(group_bcast<G>(__float_as_uint(src.l2u), pl));
        const float a2_n = __uint_as_float(group_bcast<G>(__float_as_uint(src.a2), pl));
        if constexpr (LDS_TAB) crbm_column<G, K>(s_ctab, i_n, M, gl, last_off, last_ok, cs_n);
        else crbm_column<G, K>(A.net.CS, i_n, M, gl, last_off, last_ok, cs_n);

        // proposal k: flip site i_c
        const uint32_t wbits = group_bcast<G>(word, i_c >> 5);
        const bool up = (wbits >> (i_c & 31)) & 1u;
        const float si = up ? 1.0f : -1.0f;
        float2 nn[K];
        float prod = 1.0f;
        int e2 = 0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const float4 t = cs_c[q];
            const float spx = si * t.z, spy = si * t.w;                    // s_i S
            float nx = fmaf(cc[q].x, t.x, -cc[q].y * t.y);                 // c C
            float ny = fmaf(cc[q].x, t.y, cc[q].y * t.x);
            nx = fmaf(-sh[q].x, spx, fmaf(sh[q].y, spy, nx));               // - s (s_i S)
            ny = fmaf(-sh[q].x, spy, fmaf(-sh[q].y, spx, ny));
            nn[q] = make_float2(nx, ny);
            prod *= fmaf(nx, nx, ny * ny);
            if ((q & 3) == 3 && q + 1 < K) {
                int e;
                prod = frexpf(prod, &e);
                e2 += e;
            }
        }
        const float lnew = __builtin_amdgcn_logf(prod) + (float)e2;     // log2 prod |n|^2
        const float d2 = group_sum_uniform<G>(lnew - lpart) + (up ? -a2_c : a2_c);
        const bool accept = l2u_c < d2;                                 // NaN rejects
        if (accept) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const float4 t = cs_c[q];
                const float spx = si * t.z, spy = si * t.w;
                float sx = fmaf(sh[q].x, t.x, -sh[q].y * t.y);              // s C
                float sy = fmaf(sh[q].x, t.y, sh[q].y * t.x);
                sx = fmaf(-cc[q].x, spx, fmaf(cc[q].y, spy, sx));           // - c (s_i S)
                sy = fmaf(-cc[q].x, spy, fmaf(-cc[q].y, spx, sy));
                sh[q] = make_float2(sx, sy);
                cc[q] = nn[q];
            }
            lpart = lnew;
            if (gl == (i_c >> 5)) word ^= 1u << (i_c & 31);
            ++acc;
        }
        if (traced && gl == 0) {
            const size_t idx = (size_t)c * (size_t)total + (size_t)k;
            A.tr_site[idx] = i_c | (0xFFFF << 16);
            A.tr_ubits[idx] = ub_c;
            A.tr_delta[idx] = d2 * 0.69314718055994531f;
            A.tr_acc[idx] = accept ? 1 : 0;
        }
        // advance the pipeline
        i_c = i_n;
        ub_c = ub_n;
        l2u_c = l2u_n;
        a2_c = a2_n;
        p = pn;
        if (p == G) {
            p = 0;
            base += G;
            cur = nxt;
            nxt = crbm_prop(A.net, base + G + gl, gid, A.inst, key0, key1);
        }
        if (++in_sweep == sw) {
            in_sweep = 0;
            const int64_t out = sweep - A.n_burnin;
            const bool need_f = A.logpsi != nullptr && out >= 0;
            const float f = crbm_refresh<G, K>(A.net, word, gl, cc, sh, need_f);
            lpart = 0.0f;
            if (out >= 0) {
                if (A.samples && gl < NW) {
                    int8_t *dst = A.samples + ((size_t)out * A.n_chains + c) * N + gl * 32;
                    const int nb = min(32, N - gl * 32);
                    for (int bb = 0; bb < nb; ++bb) dst[bb] = ((word >> bb) & 1u) ? 1 : -1;
                }
                if (A.logpsi && gl == 0) A.logpsi[(size_t)out * A.n_chains + c] = f;
            }
            ++sweep;
        }
    };

    int64_t k = 0;
    for (; k + 1 < total; k += 2) {
        step(k, csA, csB);
        step(k + 1, csB, csA);
    }
    if (k < total) step(k, csA, csB);

    if (gl < NW) {
        int8_t *dst = A.chain_state + (size_t)c * N + gl * 32;
        const int nb = min(32, N - gl * 32);
        for (int bb = 0; bb < nb; ++bb) dst[bb] = ((word >> bb) & 1u) ? 1 : -1;
    }
    if (A.n_acc && gl == 0) A.n_acc[c] = acc;
}

// ---- TFIM local energies, complex: B samples per workgroup ----
//
// Each table element (W for theta, (C, S) for the flip ratios) read from L2
// serves the B samples of the workgroup.  Per sample: t = tanh theta in LDS;
// one thread per site forms the complex flip ratios of all B samples,
// exp(-2 a_i s_i) prod_j (C - s_i t_j S), with frexp renormalisation every 8
// factors, and stores them in FP64; then one wave per sample sums ratios and
// diagonal bonds in a fixed order.

__device__ inline double crbm_bonds(const float *s, int i, int dim, int L, int pbc)
{
    const float si = s[i];
    double dg = 0.0;   // bonds to the right / below, each counted once
    if (dim == 1) {
        if (i + 1 < L) dg += (double)(si * s[i + 1]);
        else if (pbc) dg += (double)(si * s[0]);
    } else {
        const int x = i / L, y = i - (i / L) * L;
        if (x + 1 < L) dg += (double)(si * s[(x + 1) * L + y]);
        else if (pbc) dg += (double)(si * s[y]);
        if (y + 1 < L) dg += (double)(si * s[x * L + y + 1]);
        else if (pbc) dg += (double)(si * s[x * L]);
    }
    return dg;
}

__host__ __device__ inline size_t crbm_eloc_lds(int B, int N, int M)
{
    return sizeof(double2) * (size_t)B * N + sizeof(float2) * (size_t)B * M + sizeof(float) * (size_t)B * N;
}

template <int B>
__global__ void __launch_bounds__(256) crbm_eloc_tfim_kernel(CrbmDev net, const int8_t *__restrict__ samples,
                                                             int64_t n, int dim, int L, int pbc, double J, double h,
                                                             double *__restrict__ eloc_re, double *__restrict__ eloc_im)
{
    extern __shared__ double2 crbm_esm[];
    const int N = net.N, M = net.M, tid = threadIdx.x, nt = blockDim.x;
    double2 *rat = crbm_esm;                                             // [B][N]
    float2 *tt = reinterpret_cast<float2 *>(rat + (size_t)B * N);       // [B][M]
    float *s = reinterpret_cast<float *>(tt + (size_t)B * M);           // [B][N]
    for (int64_t k0 = (int64_t)blockIdx.x * B; k0 < n; k0 += (int64_t)gridDim.x * B) {
        const int nb = (int)(n - k0 < B ? n - k0 : B);
        for (int e = tid; e < B * N; e += nt) {
            const int bb = e / N, i = e - bb * N;
            s[e] = bb < nb ? (float)samples[(k0 + bb) * N + i] : 1.0f;
        }
        __syncthreads();
        for (int j = tid; j < M; j += nt) {
            float2 th[B];
            const float2 bj = net.b[j];
#pragma unroll
            for (int bb = 0; bb < B; ++bb) th[bb] = bj;
            for (int i = 0; i < N; ++i) {
                const float2 w = net.Wt[(int64_t)i * M + j];
#pragma unroll
                for (int bb = 0; bb < B; ++bb) {
                    const float sb = s[bb * N + i];
                    th[bb].x = fmaf(w.x, sb, th[bb].x);
                    th[bb].y = fmaf(w.y, sb, th[bb].y);
                }
            }
#pragma unroll
            for (int bb = 0; bb < B; ++bb) tt[bb * M + j] = ctanh(th[bb]);
        }
        __syncthreads();
        for (int i = tid; i < N; i += nt) {
            float2 pr[B];
            int e2[B];
            float si[B];
#pragma unroll
            for (int bb = 0; bb < B; ++bb) {
                pr[bb] = make_float2(1.0f, 0.0f);
                e2[bb] = 0;
                si[bb] = s[bb * N + i];
            }
            for (int j = 0; j < M; ++j) {
                const float4 cs = net.CSt[(int64_t)j * N + i];
#pragma unroll
                for (int bb = 0; bb < B; ++bb) {
                    const float2 ts = cmul(tt[bb * M + j], make_float2(cs.z, cs.w));
                    pr[bb] = cmul(pr[bb], make_float2(fmaf(-si[bb], ts.x, cs.x), fmaf(-si[bb], ts.y, cs.y)));
                }
                if ((j & 7) == 7) {
#pragma unroll
                    for (int bb = 0; bb < B; ++bb) {
                        int e;
                        (void)frexpf(fmaxf(fabsf(pr[bb].x), fabsf(pr[bb].y)), &e);
                        pr[bb].x = ldexpf(pr[bb].x, -e);
                        pr[bb].y = ldexpf(pr[bb].y, -e);
                        e2[bb] += e;
                    }
                }
            }
            const float2 ai = net.a[i];
#pragma unroll
            for (int bb = 0; bb < B; ++bb) {
                const double mg = exp(-2.0 * (double)ai.x * si[bb]) * ldexp(1.0, e2[bb]);
                double sn, cn;
                sincos(-2.0 * (double)ai.y * si[bb], &sn, &cn);
                const double pre = mg * cn, pim = mg * sn;
                rat[bb * N + i] = make_double2(pre * pr[bb].x - pim * pr[bb].y, pre * pr[bb].y + pim * pr[bb].x);
            }
        }
        __syncthreads();
        const int wave = tid >> 6, lane = tid & 63, nw = nt >> 6;
        for (int bb = wave; bb < nb; bb += nw) {
            double re = 0.0, im = 0.0, dg = 0.0;
            for (int i = lane; i < N; i += 64) {
                re += rat[bb * N + i].x;
                im += rat[bb * N + i].y;
                dg += crbm_bonds(s + bb * N, i, dim, L, pbc);
            }
            re = group_sum<64>(re);
            im = group_sum<64>(im);
            dg = group_sum<64>(dg);
            if (lane == 0) {
                eloc_re[k0 + bb] = J * dg + h * re;
                if (eloc_im) eloc_im[k0 + bb] = h * im;
            }
        }
        __syncthreads();
    }
}

// ---- host ----

template <int G, int K>
static void crbm_launch_gk(const CrbmSampleArgs &A, int64_t blocks, int threads, size_t lds_bytes, hipStream_t s)
{
    if (lds_bytes) {
        allow_lds(crbm_sample_kernel<G, K, true>, lds_bytes);
        hipLaunchKernelGGL((crbm_sample_kernel<G, K, true>), dim3((unsigned)blocks), dim3(threads), lds_bytes, s, A);
    } else {
        hipLaunchKernelGGL((crbm_sample_kernel<G, K, false>), dim3((unsigned)blocks), dim3(threads), 0, s, A);
    }
}

template <int G>
static void crbm_launch_g(int K, const CrbmSampleArgs &A, int64_t blocks, int threads, size_t lds_bytes, hipStream_t s)
{
    switch (K) {
    case 1: crbm_launch_gk<G, 1>(A, blocks, threads, lds_bytes, s); break;
    case 2: crbm_launch_gk<G, 2>(A, blocks, threads, lds_bytes, s); break;
    case 3: crbm_launch_gk<G, 3>(A, blocks, threads, lds_bytes, s); break;
    case 4: crbm_launch_gk<G, 4>(A, blocks, threads, lds_bytes, s); break;
    case 5: crbm_launch_gk<G, 5>(A, blocks, threads, lds_bytes, s); break;
    case 6: crbm_launch_gk<G, 6>(A, blocks, threads, lds_bytes, s); break;
    case 7: crbm_launch_gk<G, 7>(A, blocks, threads, lds_bytes, s); break;
    default: crbm_launch_gk<G, 8>(A, blocks, threads, lds_bytes, s); break;
    }
}

nqs_status crbm_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                       uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, cfg.dtype, stream);
    if (st != NQS_OK) return st;
    const CrbmDev &net = m->copies[cfg.dtype].crbm;
    const int N = net.N, M = net.M;
    // launch shape: lanes per chain G, hidden units per lane K = ceil(M / G) <= 8
    int G = cfg.lanes_per_chain;
    if (G == 0) {
        G = 16;
        while (G < 64 && ((N + 31) / 32 > G || (M + G - 1) / G > kCrbmMaxK)) G *= 2;
    } else if (G != 16 && G != 32 && G != 64) {
        return set_error(NQS_EUNSUPPORTED, "complex RBM sampler: lanes_per_chain must be 0, 16, 32 or 64");
    }
    if ((N + 31) / 32 > G) return set_error(NQS_EUNSUPPORTED, "complex RBM sampler: too many sites (N <= 32 G)");
    const int K = (M + G - 1) / G;
    if (K > kCrbmMaxK) return set_error(NQS_EUNSUPPORTED, "complex RBM sampler: at most 8 hidden units per lane (M <= 512)");
    if (cfg.init_chains) {
        st = launch_init_chains(chain_state, cfg.n_chains, N, NQS_MOVE_FLIP, cfg.seed, cfg.instance_id,
                                cfg.chain_id_offset, stream);
        if (st != NQS_OK) return st;
    }
    if (cfg.n_chains == 0) return NQS_OK;
    CrbmSampleArgs A;
    A.net = net;
    A.chain_state = chain_state;
    A.samples = samples;
    A.logpsi = logpsi;
    A.n_acc = (unsigned long long *)n_accepted;
    A.n_chains = cfg.n_chains;
    A.n_sweeps = cfg.n_sweeps;
    A.n_burnin = cfg.n_burnin;
    A.sweep_size = cfg.sweep_size > 0 ? cfg.sweep_size : N;
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
    // one LDS copy of the table per block when it fits; spread the chains over every CU
    constexpr size_t kLds = 160 * 1024;
    const size_t tab_bytes = sizeof(float4) * ((size_t)N * M + 1);
    const bool lds = tab_bytes <= kLds;
    const int max_threads = G == 16 ? 256 : 512;
    const int blocks_per_cu = lds ? (int)std::max<size_t>(1, std::min<size_t>(8, kLds / tab_bytes)) : 8;
    const int64_t slots = (int64_t)device_cus() * blocks_per_cu;
    const int cpb = (int)std::min<int64_t>(max_threads / G, std::max<int64_t>(1, (cfg.n_chains + slots - 1) / slots));
    const int64_t blocks = (cfg.n_chains + cpb - 1) / cpb;
    if (blocks > INT32_MAX) return set_error(NQS_EINVAL, "too many chains");
    const size_t lds_bytes = lds ? tab_bytes : 0;
    switch (G) {
    case 16: crbm_launch_g<16>(K, A, blocks, cpb * G, lds_bytes, stream); break;
    case 32: crbm_launch_g<32>(K, A, blocks, cpb * G, lds_bytes, stream); break;
    default: crbm_launch_g<64>(K, A, blocks, cpb * G, lds_bytes, stream); break;
    }
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status crbm_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                             double *eloc_re, double *eloc_im, hipStream_t stream)
{
    if (ham.kind != NQS_TFIM) return set_error(NQS_EUNSUPPORTED, "complex RBM local energies: TFIM");
    nqs_status st = ensure_copy(m, dtype, stream);
    if (st != NQS_OK) return st;
    const CrbmDev &net = m->copies[dtype].crbm;
    // samples per workgroup: the largest of 16, 8, 4, 2, 1 whose LDS stays within 64 KB
    int B = 16;
    while (B > 1 && crbm_eloc_lds(B, net.N, net.M) > 64 * 1024) B /= 2;
    const size_t lds = crbm_eloc_lds(B, net.N, net.M);
    if (lds > 160 * 1024) return set_error(NQS_EUNSUPPORTED, "complex RBM too large for the local-energy kernel");
    if (n == 0) return NQS_OK;
    const int threads = net.N <= 128 ? 128 : 256;
    const int64_t blocks = std::min<int64_t>((n + B - 1) / B, (int64_t)device_cus() * 8);
    switch (B) {
#define NQS_CE(BB)                                                                                                   \
    case BB:                                                                                                         \
        allow_lds(crbm_eloc_tfim_kernel<BB>, lds);                                                                   \
        hipLaunchKernelGGL(crbm_eloc_tfim_kernel<BB>, dim3((unsigned)blocks), dim3(threads), lds, stream, net,       \
                           samples, n, ham.dim, ham.L, ham.pbc, ham.J, ham.h, eloc_re, eloc_im);                     \
        break;
        NQS_CE(16) NQS_CE(8) NQS_CE(4) NQS_CE(2)
#undef NQS_CE
    default:
        allow_lds(crbm_eloc_tfim_kernel<1>, lds);
        hipLaunchKernelGGL(crbm_eloc_tfim_kernel<1>, dim3((unsigned)blocks), dim3(threads), lds, stream, net, samples,
                           n, ham.dim, ham.L, ham.pbc, ham.J, ham.h, eloc_re, eloc_im);
        break;
    }
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
