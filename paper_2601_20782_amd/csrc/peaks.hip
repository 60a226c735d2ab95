// Microbenchmarks of achievable rates (measurement support for the roofline
// figures; no step of the method runs here).  Each compute probe keeps eight
// (VALU) or four (matrix core) independent dependency chains per thread or
// wave so that issue, not latency, bounds it; a result-dependent store that
// never fires keeps the chains live.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"
#include "nqs_probe.h"

namespace nqs {

typedef float pk_f32x4 __attribute__((ext_vector_type(4)));
typedef double pk_f64x4 __attribute__((ext_vector_type(4)));
typedef short pk_s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 pk_bf16x8 __attribute__((ext_vector_type(8)));
typedef float pk_f32x16 __attribute__((ext_vector_type(16)));

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 16;

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) probe_valu_kernel(float *__restrict__ out, int iters)
{
    constexpr int kChains = KIND == NQS_PROBE_FMA_F32_DEP ? 1 : 8;
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = 1.5f + 1e-3f * (float)((t + k) & 255);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (KIND == NQS_PROBE_LOG_F32) a[k] = __builtin_amdgcn_logf(a[k]) + 2.0f;
                else if constexpr (KIND == NQS_PROBE_EXP_F32) a[k] = __builtin_amdgcn_exp2f(a[k]) * 0.25f;
                else if constexpr (KIND == NQS_PROBE_MUL_F32) a[k] = a[k] * 0.9999999f;
                else if constexpr (KIND == NQS_PROBE_DPP_ADD_F32) a[k] = a[k] + dpp_f32<0x111, 0xF, 0xF>(a[k]);
                else a[k] = fmaf(a[k], 0.9999999f, 1e-7f);   // the FMA kinds
            }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    if (s == -1.0f) out[t] = s;
}

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) probe_int_kernel(float *__restrict__ out, int iters)
{
    const uint32_t t = blockIdx.x * kProbeThreads + threadIdx.x;
    uint32_t a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0x9E3779B9u * (t + (uint32_t)k) + 1u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if constexpr (KIND == NQS_PROBE_MULHI_U32) a[k] = __umulhi(a[k], 0xD2511F53u);
                else asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[k]) : "v"(a[(k + 1) & 7]));   // kept as written
            }
    }
    uint32_t s = 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) s ^= a[k];
    if (s == 0x12345678u) out[t] = (float)s;
}

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) probe_mfma_kernel(float *__restrict__ out, int iters)
{
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    const float v = 1e-3f * (float)(t & 63);
    float s = 0.0f;
    if constexpr (KIND == NQS_PROBE_MFMA_F64) {
        pk_f64x4 acc[4] = {};
        const double a = v, b = 1.0 - v;
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) s += (float)(acc[k][0] + acc[k][3]);
    } else {
        pk_f32x4 acc[4] = {};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if constexpr (KIND == NQS_PROBE_MFMA_F32) {
                        acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(v, 1.0f - v, acc[k], 0, 0, 0);
                    } else if constexpr (KIND == NQS_PROBE_MFMA_BF16_K16) {
                        const short c = (short)(__float_as_uint(v) >> 16);
                        const pk_s16x4 a = {c, c, c, c};
                        acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, a, acc[k], 0, 0, 0);
                    } else {
                        const __bf16 c = (__bf16)v;
                        const pk_bf16x8 a = {c, c, c, c, c, c, c, c};
                        acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[k], 0, 0, 0);
                    }
                }
#pragma unroll
        for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][3];
    }
    if (s == -1.0f) out[t] = s;
}

// One block of 512 threads per compute unit: LDS reads (KIND = LDS_READ), or one chain of 32 x 32 x 16 products per
// wave with B from registers or from LDS (row lane % 32, columns 16 k + 8 (lane / 32) of a 32 x 512 tile whose
// rows are padded by 8 values so that the 32 rows of a read fall in different banks; for _LDS each B read is issued
// two products ahead of its use, the order pinned against the scheduler, for _LDS_JIT the compiler places them).  The offset of each iteration goes through an empty asm statement so that the
// compiler cannot prove two iterations read the same words.
constexpr int kProbeLdsThreads = 512;
constexpr int kProbeLdsCols = 512;
constexpr int kProbeLdsLd = kProbeLdsCols + 8;

template <int KIND>
__global__ void __launch_bounds__(kProbeLdsThreads) probe_lds_kernel(float *__restrict__ out, int iters)
{
    __shared__ __align__(16) __bf16 tile[32 * kProbeLdsLd];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int k = tid; k < 32 * kProbeLdsLd; k += kProbeLdsThreads) tile[k] = (__bf16)(1e-3f * (float)(k & 127));
    __syncthreads();
    float s = 0.0f;
    if constexpr (KIND == NQS_PROBE_LDS_READ) {
        // lane l reads word l + 64 m, m = (offset + u + wave) mod 32: consecutive lanes, consecutive words
        const uint4 *w = reinterpret_cast<const uint4 *>(tile);
        uint32_t x = 0u;
        for (int it = 0; it < iters; ++it) {
            int o = it * kProbeUnroll + (tid >> 6);
            asm volatile("" : "+v"(o));
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) {
                const uint4 v = w[lane + 64 * ((o + u) & 31)];
                x += (v.x ^ v.y) + (v.z ^ v.w);
            }
        }
        if (x == 0x12345678u) out[blockIdx.x * kProbeLdsThreads + tid] = 1.0f;
    } else {
        const pk_bf16x8 a = {(__bf16)1e-3f, (__bf16)2e-3f, (__bf16)3e-3f, (__bf16)4e-3f,
                             (__bf16)5e-3f, (__bf16)6e-3f, (__bf16)7e-3f, (__bf16)8e-3f};
        pk_f32x16 acc = {};
        const __bf16 *row = tile + (lane & 31) * kProbeLdsLd + 8 * (lane >> 5);
        for (int it = 0; it < iters; ++it) {
            if constexpr (KIND == NQS_PROBE_MFMA_BF16_32_LDS_JIT) {
                int o = it * kProbeUnroll;
                asm volatile("" : "+v"(o));
#pragma unroll
                for (int u = 0; u < kProbeUnroll; ++u) {
                    const pk_bf16x8 b = *reinterpret_cast<const pk_bf16x8 *>(row + 16 * ((o + u) & 31));
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
                }
            } else if constexpr (KIND == NQS_PROBE_MFMA_BF16_32_LDS) {
                int o = it * kProbeUnroll;
                asm volatile("" : "+v"(o));
                pk_bf16x8 b[kProbeUnroll];
                b[0] = *reinterpret_cast<const pk_bf16x8 *>(row + 16 * (o & 31));
                b[1] = *reinterpret_cast<const pk_bf16x8 *>(row + 16 * ((o + 1) & 31));
#pragma unroll
                for (int u = 0; u < kProbeUnroll; ++u) {
                    if (u + 2 < kProbeUnroll) b[u + 2] = *reinterpret_cast<const pk_bf16x8 *>(row + 16 * ((o + u + 2) & 31));
                    __builtin_amdgcn_sched_barrier(0);   // keep each read two products ahead of its use
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[u], acc, 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int u = 0; u < kProbeUnroll; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, acc, 0, 0, 0);
            }
        }
        s = acc[0] + acc[15];
    }
    if (s == -1.0f) out[blockIdx.x * kProbeLdsThreads + tid] = s;
}

__global__ void __launch_bounds__(kProbeThreads) probe_read_kernel(const float4 *__restrict__ src, int64_t n4,
                                                                   float *__restrict__ out)
{
    float s = 0.0f;
    for (int64_t k = blockIdx.x * (int64_t)kProbeThreads + threadIdx.x; k < n4;
         k += (int64_t)gridDim.x * kProbeThreads) {
        const float4 v = src[k];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == -1.0f) out[blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kProbeThreads) probe_copy_kernel(const float4 *__restrict__ src, int64_t n4,
                                                                   float4 *__restrict__ dst)
{
    for (int64_t k = blockIdx.x * (int64_t)kProbeThreads + threadIdx.x; k < n4;
         k += (int64_t)gridDim.x * kProbeThreads)
        dst[k] = src[k];
}

}  // namespace nqs

using namespace nqs;

extern "C" nqs_status nqs_probe_rate(int32_t kind, int64_t size, const void *src, void *dst, double *work,
                                     void *stream)
{
    if (!work) return set_error(NQS_EINVAL, "NULL work");
    const bool compute = (kind >= NQS_PROBE_FMA_F32 && kind <= NQS_PROBE_MFMA_F64) ||
                         (kind >= NQS_PROBE_MUL_F32 && kind <= NQS_PROBE_MFMA_BF16_32_LDS_JIT);
    const bool memory = kind == NQS_PROBE_HBM_READ || kind == NQS_PROBE_HBM_COPY;
    if (!compute && !memory) return set_error(NQS_EINVAL, "unknown probe kind");
    if (compute && (size < 1 || size > (1 << 24))) return set_error(NQS_EINVAL, "iterations must be in [1, 2^24]");
    if (compute && !dst) return set_error(NQS_EINVAL, "NULL scratch");
    if (memory) {
        if (size <= 0 || size % 16 != 0) return set_error(NQS_EINVAL, "size must be a positive multiple of 16");
        if (!src || ((uintptr_t)src & 15)) return set_error(NQS_EINVAL, "src must be 16-byte aligned");
        if (!dst || ((uintptr_t)dst & 15)) return set_error(NQS_EINVAL, "dst must be 16-byte aligned");
    }
    hipStream_t s = (hipStream_t)stream;
    const int blocks = device_cus() * 8;
    const double threads = (double)blocks * kProbeThreads;
    if (compute) {
        float *o = (float *)dst;
        const int it = (int)size;
        const double per = (double)it * kProbeUnroll;
        switch (kind) {
        case NQS_PROBE_FMA_F32:
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_FMA_F32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8 * 2;
            break;
        case NQS_PROBE_LOG_F32:
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_LOG_F32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8;
            break;
        case NQS_PROBE_EXP_F32:
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_EXP_F32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8;
            break;
        case NQS_PROBE_MUL_F32:
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_MUL_F32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8;
            break;
        case NQS_PROBE_DPP_ADD_F32:
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_DPP_ADD_F32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8;
            break;
        case NQS_PROBE_XOR_U32:
            hipLaunchKernelGGL(probe_int_kernel<NQS_PROBE_XOR_U32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8;
            break;
        case NQS_PROBE_MULHI_U32:
            hipLaunchKernelGGL(probe_int_kernel<NQS_PROBE_MULHI_U32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads * per * 8;
            break;
        case NQS_PROBE_FMA_F32_W1:
        case NQS_PROBE_FMA_F32_W2: {
            const int b = device_cus() * (kind == NQS_PROBE_FMA_F32_W1 ? 1 : 2);
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_FMA_F32_W1>, dim3(b), dim3(kProbeThreads), 0, s, o, it);
            *work = (double)b * kProbeThreads * per * 8 * 2;
            break;
        }
        case NQS_PROBE_FMA_F32_DEP: {
            const int b = device_cus();
            hipLaunchKernelGGL(probe_valu_kernel<NQS_PROBE_FMA_F32_DEP>, dim3(b), dim3(kProbeThreads), 0, s, o, it);
            *work = (double)b * kProbeThreads * per * 2;
            break;
        }
        case NQS_PROBE_LDS_READ:
            hipLaunchKernelGGL(probe_lds_kernel<NQS_PROBE_LDS_READ>, dim3(device_cus()), dim3(kProbeLdsThreads), 0, s,
                               o, it);
            *work = (double)device_cus() * kProbeLdsThreads * per * 16;
            break;
        case NQS_PROBE_MFMA_BF16_32:
            hipLaunchKernelGGL(probe_lds_kernel<NQS_PROBE_MFMA_BF16_32>, dim3(device_cus()), dim3(kProbeLdsThreads), 0,
                               s, o, it);
            *work = (double)device_cus() * (kProbeLdsThreads / 64) * per * (2.0 * 32 * 32 * 16);
            break;
        case NQS_PROBE_MFMA_BF16_32_LDS:
            hipLaunchKernelGGL(probe_lds_kernel<NQS_PROBE_MFMA_BF16_32_LDS>, dim3(device_cus()),
                               dim3(kProbeLdsThreads), 0, s, o, it);
            *work = (double)device_cus() * (kProbeLdsThreads / 64) * per * (2.0 * 32 * 32 * 16);
            break;
        case NQS_PROBE_MFMA_BF16_32_LDS_JIT:
            hipLaunchKernelGGL(probe_lds_kernel<NQS_PROBE_MFMA_BF16_32_LDS_JIT>, dim3(device_cus()),
                               dim3(kProbeLdsThreads), 0, s, o, it);
            *work = (double)device_cus() * (kProbeLdsThreads / 64) * per * (2.0 * 32 * 32 * 16);
            break;
        case NQS_PROBE_MFMA_BF16_K16:
            hipLaunchKernelGGL(probe_mfma_kernel<NQS_PROBE_MFMA_BF16_K16>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads / 64 * per * 4 * (2.0 * 16 * 16 * 16);
            break;
        case NQS_PROBE_MFMA_BF16_K32:
            hipLaunchKernelGGL(probe_mfma_kernel<NQS_PROBE_MFMA_BF16_K32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads / 64 * per * 4 * (2.0 * 16 * 16 * 32);
            break;
        case NQS_PROBE_MFMA_F32:
            hipLaunchKernelGGL(probe_mfma_kernel<NQS_PROBE_MFMA_F32>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads / 64 * per * 4 * (2.0 * 16 * 16 * 4);
            break;
        default:
            hipLaunchKernelGGL(probe_mfma_kernel<NQS_PROBE_MFMA_F64>, dim3(blocks), dim3(kProbeThreads), 0, s, o, it);
            *work = threads / 64 * per * 4 * (2.0 * 16 * 16 * 4);
            break;
        }
    } else {
        const int64_t n4 = size / 16;
        const int mb = blocks * 2;
        if (kind == NQS_PROBE_HBM_READ) {
            hipLaunchKernelGGL(probe_read_kernel, dim3(mb), dim3(kProbeThreads), 0, s, (const float4 *)src, n4,
                               (float *)dst);
            *work = (double)size;
        } else {
            hipLaunchKernelGGL(probe_copy_kernel, dim3(mb), dim3(kProbeThreads), 0, s, (const float4 *)src, n4,
                               (float4 *)dst);
            *work = 2.0 * (double)size;
        }
    }
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}
