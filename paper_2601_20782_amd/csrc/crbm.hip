// Complex-parameter RBM: log psi = sum_i a_i s_i + sum_j log cosh(theta_j),
// theta = W s + b, a, b, W complex; the sampled distribution is |psi|^2 =
// exp(2 Re log psi).  Flipping site i multiplies psi by
//     exp(-2 a_i s_i) prod_j (C_ji - s_i t_j S_ji),
// C = cosh 2W, S = sinh 2W, t = tanh theta (all complex).
//
// Sampler: one wave per chain, lanes over hidden units; each lane keeps theta_j
// and t_j of its units (FP32 complex), updates theta on acceptance and takes
// t = tanh theta afresh; theta is recomputed from W s + b every sweep.  The
// acceptance log-ratio is -4 Re(a_i) s_i + sum_j log |C - s t S|^2.
// Local energies: one sample per workgroup, one thread per site, the complex
// flip ratios summed in FP64 (real and imaginary parts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
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
    const size_t bytes = al(sizeof(float2) * N) + al(sizeof(float2) * M) + al(sizeof(float2) * nm) +
                         2 * al(sizeof(float4) * nm);
    if (!c.block) NQS_HIP_TRY(hipMalloc(&c.block, bytes));
    char *p = (char *)c.block;
    d.a = (float2 *)p;
    p += al(sizeof(float2) * N);
    d.b = (float2 *)p;
    p += al(sizeof(float2) * M);
    d.Wt = (float2 *)p;
    p += al(sizeof(float2) * nm);
    d.CS = (float4 *)p;
    p += al(sizeof(float4) * nm);
    d.CSt = (float4 *)p;
    const int64_t P = N + M + (int64_t)nm;
    hipLaunchKernelGGL(crbm_build_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, m->master, N, M,
                       dtype, d);
    NQS_HIP_TRY(hipGetLastError());
    c.valid = true;
    return NQS_OK;
}

// ---- complex helpers (FP32) ----

__device__ inline float2 cmul(float2 x, float2 y) { return make_float2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x); }

// tanh(x + iy) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y)
__device__ inline float2 ctanh(float2 z)
{
    const float ax = fminf(fabsf(2.0f * z.x), 80.0f);
    const float e = __expf(ax), ei = 1.0f / e;
    const float ch = 0.5f * (e + ei), sh = copysignf(0.5f * (e - ei), z.x);
    float sy, cy;
    sincosf(2.0f * z.y, &sy, &cy);
    const float den = ch + cy;
    return make_float2(sh / den, sy / den);
}

// log |cosh(x + iy)| = 0.5 log((cosh 2x + cos 2y) / 2)
__device__ inline float clogcosh_re(float2 z)
{
    const float ax = fabsf(2.0f * z.x);
    // cosh 2x + cos 2y = e^{|2x|} (1 + e^{-2|2x|}) / 2 + cos 2y
    const float e = __expf(-ax);
    const float v = 0.5f * (1.0f + e * e) + cosf(2.0f * z.y) * e;
    return 0.5f * (ax + logf(v)) - 0.5f * 0.6931471805599453f;
}

// ---- sampler: one wave per chain ----

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

template <int K>
__device__ inline void crbm_refresh(const CrbmDev &net, const float *s, int lane, float2 (&th)[K], float2 (&t)[K])
{
    const int N = net.N, M = net.M;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int j = lane + 64 * q;
        float2 a = j < M ? net.b[j] : make_float2(0.0f, 0.0f);
        if (j < M)
            for (int i = 0; i < N; ++i) {
                const float2 w = net.Wt[(int64_t)i * M + j];
                a.x = fmaf(w.x, s[i], a.x);
                a.y = fmaf(w.y, s[i], a.y);
            }
        th[q] = a;
        t[q] = ctanh(a);
    }
}

template <int K>
__global__ void __launch_bounds__(kCrbmThreads) crbm_sample_kernel(CrbmSampleArgs A)
{
    extern __shared__ float csm[];
    const int N = A.net.N, M = A.net.M;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *s = csm + (size_t)wave * N;
    const uint32_t key0 = (uint32_t)A.seed, key1 = (uint32_t)(A.seed >> 32);
    const int64_t total = (int64_t)(A.n_burnin + A.n_sweeps) * A.sweep_size;
    for (int64_t c = (int64_t)blockIdx.x * (kCrbmThreads / 64) + wave; c < A.n_chains;
         c += (int64_t)gridDim.x * (kCrbmThreads / 64)) {
        const uint32_t gid = A.chain_id_offset + (uint32_t)c;
        for (int i = lane; i < N; i += 64) s[i] = (float)A.chain_state[c * N + i];
        __builtin_amdgcn_wave_barrier();
        float2 th[K], t[K];
        crbm_refresh<K>(A.net, s, lane, th, t);
        unsigned long long acc = 0;
        for (int64_t k = 0; k < total; ++k) {
            const uint64_t step = A.step_offset + (uint64_t)k;
            const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, A.inst << 8, key0, key1);
            const int i = index_from_word(rb.r0, N);
            const uint32_t ub = rb.r2 >> 8;
            const float si = s[i];
            float part = 0.0f;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int j = lane + 64 * q;
                if (j < M) {
                    const float4 cs = A.net.CS[(int64_t)i * M + j];
                    const float2 ts = cmul(t[q], make_float2(cs.z, cs.w));
                    const float2 r = make_float2(fmaf(-si, ts.x, cs.x), fmaf(-si, ts.y, cs.y));
                    part += __logf(fmaf(r.x, r.x, r.y * r.y));
                }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
            const float d = fmaf(-4.0f * A.net.a[i].x, si, part);            // ln |psi(s')/psi(s)|^2
            const float lu = __logf((float)ub * 5.9604644775390625e-8f);     // ln u
            const bool accept = lu < d;                                      // NaN rejects
            if (accept) {
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const int j = lane + 64 * q;
                    if (j < M) {
                        const float2 w = A.net.Wt[(int64_t)i * M + j];
                        th[q].x = fmaf(-2.0f * si, w.x, th[q].x);
                        th[q].y = fmaf(-2.0f * si, w.y, th[q].y);
                        t[q] = ctanh(th[q]);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) s[i] = -si;
                __builtin_amdgcn_wave_barrier();
                ++acc;
            }
            if (c < A.n_traced && lane == 0) {
                const size_t idx = (size_t)c * (size_t)total + (size_t)k;
                A.tr_site[idx] = i | (0xFFFF << 16);
                A.tr_ubits[idx] = ub;
                A.tr_delta[idx] = d;
                A.tr_acc[idx] = accept ? 1 : 0;
            }
            if ((k + 1) % A.sweep_size == 0) {
                crbm_refresh<K>(A.net, s, lane, th, t);
                const int64_t out = (k + 1) / A.sweep_size - 1 - A.n_burnin;
                if (out >= 0) {
                    if (A.samples)
                        for (int ii = lane; ii < N; ii += 64)
                            A.samples[((size_t)out * A.n_chains + c) * N + ii] = s[ii] > 0.0f ? 1 : -1;
                    if (A.logpsi) {
                        float lr = 0.0f;
#pragma unroll
                        for (int q = 0; q < K; ++q)
                            if (lane + 64 * q < M) lr += clogcosh_re(th[q]);
                        for (int ii = lane; ii < N; ii += 64) lr = fmaf(A.net.a[ii].x, s[ii], lr);
#pragma unroll
                        for (int o = 32; o >= 1; o >>= 1) lr += __shfl_xor(lr, o, 64);
                        if (lane == 0) A.logpsi[(size_t)out * A.n_chains + c] = lr;
                    }
                }
            }
        }
        for (int i = lane; i < N; i += 64) A.chain_state[c * N + i] = s[i] > 0.0f ? 1 : -1;
        if (A.n_acc && lane == 0) A.n_acc[c] = acc;
        __builtin_amdgcn_wave_barrier();
    }
}

// ---- TFIM local energies, complex: one sample per workgroup ----

__global__ void __launch_bounds__(kCrbmThreads) crbm_eloc_tfim_kernel(CrbmDev net, const int8_t *__restrict__ samples,
                                                                      int64_t n, int dim, int L, int pbc, double J,
                                                                      double h, double *__restrict__ eloc_re,
                                                                      double *__restrict__ eloc_im)
{
    extern __shared__ float esm[];
    const int N = net.N, M = net.M, tid = threadIdx.x;
    float *s = esm;                                          // [N]
    float2 *tt = reinterpret_cast<float2 *>(esm + ((N + 1) & ~1));   // [M]
    __shared__ double red[3][kCrbmThreads / 64];
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        for (int i = tid; i < N; i += kCrbmThreads) s[i] = (float)samples[k * N + i];
        __syncthreads();
        for (int j = tid; j < M; j += kCrbmThreads) {
            float2 a = net.b[j];
            for (int i = 0; i < N; ++i) {
                const float2 w = net.Wt[(int64_t)i * M + j];
                a.x = fmaf(w.x, s[i], a.x);
                a.y = fmaf(w.y, s[i], a.y);
            }
            tt[j] = ctanh(a);
        }
        __syncthreads();
        double re = 0.0, im = 0.0, dg = 0.0;
        for (int i = tid; i < N; i += kCrbmThreads) {
            const float si = s[i];
            // ratio = exp(-2 a_i s_i) prod_j (C - s_i t_j S), magnitudes renormalised every 8 factors
            float2 pr = make_float2(1.0f, 0.0f);
            int e2 = 0;
            for (int j = 0; j < M; ++j) {
                const float4 cs = net.CSt[(int64_t)j * N + i];
                const float2 ts = cmul(tt[j], make_float2(cs.z, cs.w));
                pr = cmul(pr, make_float2(fmaf(-si, ts.x, cs.x), fmaf(-si, ts.y, cs.y)));
                if ((j & 7) == 7) {
                    int e;
                    const float mag = frexpf(fmaxf(fabsf(pr.x), fabsf(pr.y)), &e);
                    (void)mag;
                    pr.x = ldexpf(pr.x, -e);
                    pr.y = ldexpf(pr.y, -e);
                    e2 += e;
                }
            }
            const float2 ai = net.a[i];
            const double mg = exp(-2.0 * (double)ai.x * si) * ldexp(1.0, e2);
            double sn, cn;
            sincos(-2.0 * (double)ai.y * si, &sn, &cn);
            const double pre = mg * cn, pim = mg * sn;
            re += pre * pr.x - pim * pr.y;
            im += pre * pr.y + pim * pr.x;
            // bonds to the right / below, each counted once
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
        }
        re = group_sum<64>(re);
        im = group_sum<64>(im);
        dg = group_sum<64>(dg);
        if ((tid & 63) == 0) {
            red[0][tid >> 6] = re;
            red[1][tid >> 6] = im;
            red[2][tid >> 6] = dg;
        }
        __syncthreads();
        if (tid == 0) {
            double R = 0.0, I = 0.0, D = 0.0;
            for (int w = 0; w < kCrbmThreads / 64; ++w) {
                R += red[0][w];
                I += red[1][w];
                D += red[2][w];
            }
            eloc_re[k] = J * D + h * R;
            if (eloc_im) eloc_im[k] = h * I;
        }
        __syncthreads();
    }
}

// ---- host ----

nqs_status crbm_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                       uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream)
{
    nqs_status st = ensure_copy(m, cfg.dtype, stream);
    if (st != NQS_OK) return st;
    const CrbmDev &net = m->copies[cfg.dtype].crbm;
    const int N = net.N, M = net.M;
    const int K = (M + 63) / 64;
    if (K > 8) return set_error(NQS_EUNSUPPORTED, "complex RBM sampler: at most 512 hidden units");
    if (cfg.init_chains) {
        st = launch_init_chains(chain_state, cfg.n_chains, N, NQS_MOVE_FLIP, cfg.seed, cfg.instance_id,
                                cfg.chain_id_offset, stream);
        if (st != NQS_OK) return st;
    }
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
    const size_t lds = sizeof(float) * (size_t)N * (kCrbmThreads / 64);
    const int64_t blocks =
        std::min<int64_t>((cfg.n_chains + kCrbmThreads / 64 - 1) / (kCrbmThreads / 64), (int64_t)device_cus() * 16);
    switch (K) {
#define NQS_CK(KK)                                                                                                   \
    case KK:                                                                                                         \
        hipLaunchKernelGGL(crbm_sample_kernel<KK>, dim3((unsigned)blocks), dim3(kCrbmThreads), lds, stream, A);      \
        break;
        NQS_CK(1) NQS_CK(2) NQS_CK(3) NQS_CK(4) NQS_CK(5) NQS_CK(6) NQS_CK(7) NQS_CK(8)
#undef NQS_CK
    default: break;
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
    const size_t lds = sizeof(float) * (((size_t)net.N + 1) & ~(size_t)1) + sizeof(float2) * (size_t)net.M;
    if (lds > 160 * 1024) return set_error(NQS_EUNSUPPORTED, "complex RBM too large for the local-energy kernel");
    allow_lds(crbm_eloc_tfim_kernel, lds);
    const int64_t blocks = std::min<int64_t>(n, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(crbm_eloc_tfim_kernel, dim3((unsigned)blocks), dim3(kCrbmThreads), lds, stream, net, samples, n,
                       ham.dim, ham.L, ham.pbc, ham.J, ham.h, eloc_re, eloc_im);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
