// Downcast, chain initialisation and the FP64 averages (energy statistics, forces).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "common.h"
#include "internal.h"

namespace nqs {

// ---------------------------------------------------------------------------
// Downcast of the FP64 master (two-copy scheme, Sec. IV.B; formats of App. A).
// ---------------------------------------------------------------------------
__global__ void amax_kernel(const double *__restrict__ x, int64_t n, unsigned long long *amax_bits)
{
    double m = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(x[k]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(amax_bits, (unsigned long long)__double_as_longlong(m));
}

// scale = amax / 448 rounded to FP32 (1 when the tensor is all zeros)
__device__ __forceinline__ float e4m3_scale_from_bits(unsigned long long bits)
{
    const double amax = __longlong_as_double((long long)bits);
    return amax > 0.0 ? (float)(amax / 448.0) : 1.0f;
}

__global__ void downcast_kernel(const double *__restrict__ src, int64_t n, int dtype, float *__restrict__ dst,
                                const unsigned long long *amax_bits, float *scale_out)
{
    float scale = 1.0f;
    if (dtype == kE4M3) {
        scale = e4m3_scale_from_bits(*amax_bits);
        if (scale_out && blockIdx.x == 0 && threadIdx.x == 0) *scale_out = scale;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        if (dtype == kE4M3) {
            const double q = round_to_dtype(src[k] / (double)scale, kE4M3);
            dst[k] = (float)(q * (double)scale);
        } else {
            dst[k] = (float)round_to_dtype(src[k], dtype);
        }
    }
}

nqs_status launch_downcast(const double *src, int64_t n, int dtype, float *dst, float *scale_out, hipStream_t stream)
{
    unsigned long long *amax = nullptr;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    if (dtype == kE4M3) {
        amax = (unsigned long long *)workspace(256, stream);
        if (!amax) return set_error(NQS_ENOMEM, "workspace allocation failed");
        if (nqs_status z = launch_zero_u64(amax, 1, stream); z != NQS_OK) return z;
        hipLaunchKernelGGL(amax_kernel, dim3(std::min(blocks, 1024)), dim3(256), 0, stream, src, n, amax);
        NQS_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(downcast_kernel, dim3(blocks), dim3(256), 0, stream, src, n, dtype, dst, amax, scale_out);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// Initial chain states from the init stream (counter tag 1); word w of a
// chain's stream is component w%4 of block w/4.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t init_word(uint64_t seed, uint32_t chain, uint32_t inst, uint32_t w)
{
    const Block4 b = stream_block(seed, (uint64_t)(w >> 2), chain, inst, 1u);
    switch (w & 3u) {
    case 0: return b.r0;
    case 1: return b.r1;
    case 2: return b.r2;
    default: return b.r3;
    }
}

__global__ void init_chains_kernel(int8_t *__restrict__ state, int64_t n_chains, int N, int move, uint64_t seed,
                                   uint32_t inst, uint32_t chain_id_offset)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n_chains) return;
    const uint32_t gid = chain_id_offset + (uint32_t)c;
    int8_t *s = state + c * N;
    if (move == NQS_MOVE_FLIP) {
        for (int w = 0; w * 32 < N; ++w) {
            const uint32_t bits = init_word(seed, gid, inst, (uint32_t)w);
            const int nb = min(32, N - 32 * w);
            for (int b = 0; b < nb; ++b) s[32 * w + b] = ((bits >> b) & 1u) ? 1 : -1;
        }
    } else {
        // Fisher-Yates over N/2 up and N/2 down spins
        for (int i = 0; i < N; ++i) s[i] = i < N / 2 ? 1 : -1;
        for (int k = N - 1; k >= 1; --k) {
            const uint32_t r = init_word(seed, gid, inst, (uint32_t)(N - 1 - k));
            const int j = index_from_word(r, k + 1);
            const int8_t t = s[k];
            s[k] = s[j];
            s[j] = t;
        }
    }
}

// Zero fill by a kernel (not hipMemsetAsync), so that the call can sit in a captured graph.
__global__ void zero_u64_kernel(unsigned long long *p, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0ull;
}

// One tensor of an FP8 copy: scale = amax / 448 (FP32), values round(x / scale) * scale.
// `amax` is one 64-bit word of caller-owned device memory.
nqs_status launch_e4m3_tensor(const double *src, int64_t n, unsigned long long *amax, float *dst, hipStream_t stream)
{
    if (n <= 0) return NQS_OK;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, amax, (int64_t)1);
    hipLaunchKernelGGL(amax_kernel, dim3(std::min(blocks, 1024)), dim3(256), 0, stream, src, n, amax);
    hipLaunchKernelGGL(downcast_kernel, dim3(blocks), dim3(256), 0, stream, src, n, (int)kE4M3, dst,
                       (const unsigned long long *)amax, (float *)nullptr);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status launch_zero_u64(void *p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return NQS_OK;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(blocks), dim3(256), 0, stream, (unsigned long long *)p, n);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status launch_init_chains(int8_t *chain_state, int64_t n_chains, int N, int move, uint64_t seed, uint32_t inst,
                              int64_t chain_id_offset, hipStream_t stream)
{
    const int64_t blocks = (n_chains + 127) / 128;
    hipLaunchKernelGGL(init_chains_kernel, dim3((unsigned)blocks), dim3(128), 0, stream, chain_state, n_chains, N, move,
                       seed, inst, (uint32_t)chain_id_offset);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// FP64 statistics of the local energies (Eq. eq:loss): mean, unbiased
// variance, standard error of the per-chain means (layout [sweep][chain]).
// Fixed reduction trees: the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 512;

// partial[b] = sum over the block's slice of (x - shift)^power, shift = shift_src ? *shift_src : 0
__global__ void __launch_bounds__(256) moment_partial_kernel(const double *__restrict__ x, int64_t n,
                                                             const double *shift_src, int power,
                                                             double *__restrict__ partial)
{
    __shared__ double red[4];
    const double shift = shift_src ? *shift_src : 0.0;
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const double d = x[k] - shift;
        acc += power == 1 ? d : d * d;
    }
    acc = group_sum<64>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out[slot] = transform(sum of partial[0..nb))
__global__ void __launch_bounds__(256) finalize_kernel(const double *__restrict__ partial, int nb, int mode,
                                                       double count, double *stats)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) acc += partial[k];
    acc = group_sum<64>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double s = red[0] + red[1] + red[2] + red[3];
    if (mode == 0) stats[0] = s / count;                                      // mean
    else if (mode == 1) stats[1] = count > 1 ? s / (count - 1.0) : 0.0;       // variance
    else stats[2] = count > 1 ? sqrt(s / (count - 1.0) / count) : 0.0;        // stderr of chain means
}

__global__ void chain_means_kernel(const double *__restrict__ x, int64_t per, int64_t C, double *__restrict__ out)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int64_t t = 0; t < per; ++t) s += x[t * C + c];
    out[c] = s / (double)per;
}

__global__ void set_tail_kernel(double *stats, double n, int valid_se)
{
    if (!valid_se) stats[2] = __longlong_as_double(0x7FF8000000000000ll);
    stats[3] = n;
}

// The statistics with caller-chosen scratch `ws` of at least energy_stats_scratch_doubles(n, n_chains)
// doubles: block partials, then the chain means.  Every slot is written before it is read, so the
// scratch needs no clearing.
static size_t energy_stats_scratch_doubles(int64_t n, int64_t n_chains)
{
    const bool se = n_chains >= 2 && n % n_chains == 0;
    return (size_t)kRedBlocks + (se ? (size_t)n_chains : 0);
}

static nqs_status energy_stats_with(const double *eloc, int64_t n, int64_t n_chains, double *stats, double *ws,
                                    hipStream_t stream)
{
    const bool se = n_chains >= 2 && n % n_chains == 0;
    double *partial = ws, *cm = ws + kRedBlocks;
    const int nb = (int)std::min<int64_t>(kRedBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(moment_partial_kernel, dim3(nb), dim3(256), 0, stream, eloc, n, (const double *)nullptr, 1, partial);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, stream, partial, nb, 0, (double)n, stats);
    hipLaunchKernelGGL(moment_partial_kernel, dim3(nb), dim3(256), 0, stream, eloc, n, (const double *)stats, 2, partial);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, stream, partial, nb, 1, (double)n, stats);
    if (se) {
        const int64_t per = n / n_chains;
        hipLaunchKernelGGL(chain_means_kernel, dim3((unsigned)((n_chains + 255) / 256)), dim3(256), 0, stream, eloc, per,
                           n_chains, cm);
        const int nb2 = (int)std::min<int64_t>(kRedBlocks, (n_chains + 255) / 256);
        hipLaunchKernelGGL(moment_partial_kernel, dim3(nb2), dim3(256), 0, stream, (const double *)cm, n_chains,
                           (const double *)stats, 2, partial);
        hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, stream, partial, nb2, 2, (double)n_chains, stats);
    }
    hipLaunchKernelGGL(set_tail_kernel, dim3(1), dim3(1), 0, stream, stats, (double)n, se ? 1 : 0);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

nqs_status launch_energy_stats(const double *eloc, int64_t n, int64_t n_chains, double *stats, hipStream_t stream)
{
    double *ws = (double *)workspace(sizeof(double) * energy_stats_scratch_doubles(n, n_chains), stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    return energy_stats_with(eloc, n, n_chains, stats, ws, stream);
}

// ---------------------------------------------------------------------------
// The same statistics without any allocation, for callers that cannot
// allocate (graph capture, serving loops): the scratch is a file-scope device
// array, one copy per GPU, held until the process ends.  Host code never
// names the array: its device address is looked up once per device with
// hipGetSymbolAddress (the device current) and kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kStatsScratchDoubles];

constexpr int kMaxDevices = 64;
static double *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mutex;

static nqs_status stats_scratch(double **out)
{
    int dev = 0;
    NQS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(NQS_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        NQS_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(NQS_EDEVICE, "no device address for the statistics scratch");
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return NQS_OK;
}

nqs_status launch_energy_stats_noalloc(const double *eloc, int64_t n, int64_t n_chains, double *stats,
                                       hipStream_t stream)
{
    if (energy_stats_scratch_doubles(n, n_chains) > (size_t)kStatsScratchDoubles)
        return set_error(NQS_EINVAL, "n_chains exceeds the static scratch of nqs_energy_stats_noalloc (at most " +
                                         std::to_string(kStatsScratchDoubles - kRedBlocks) + " chains)");
    double *ws = nullptr;
    nqs_status st = stats_scratch(&ws);
    if (st != NQS_OK) return st;
    return energy_stats_with(eloc, n, n_chains, stats, ws, stream);
}

// ---------------------------------------------------------------------------
// Forces F = E[O eps] - E[O] E[eps] (Eq. eq:forces), FP64 accumulation.
// A block covers 256 consecutive parameters and a slice of samples; slices
// are combined in a fixed order by a second pass.
// ---------------------------------------------------------------------------
constexpr int kForceSlices = 64;

__global__ void __launch_bounds__(256) forces_partial_kernel(const float *__restrict__ O, const double *__restrict__ e,
                                                             int64_t n, int64_t P, int64_t per_slice,
                                                             double *__restrict__ part_oe, double *__restrict__ part_o,
                                                             double *__restrict__ part_e)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int slice = blockIdx.y;
    const int64_t k0 = slice * per_slice, k1 = min(n, k0 + per_slice);
    double oe = 0.0, o = 0.0, es = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        const double ek = e[k];
        es += ek;
        if (p < P) {
            const double v = (double)O[k * P + p];
            oe = fma(v, ek, oe);
            o += v;
        }
    }
    if (p < P) {
        part_oe[(int64_t)slice * P + p] = oe;
        part_o[(int64_t)slice * P + p] = o;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) part_e[slice] = es;
}

__global__ void forces_final_kernel(const double *__restrict__ part_oe, const double *__restrict__ part_o,
                                    const double *__restrict__ part_e, int slices, int64_t n, int64_t P,
                                    double *__restrict__ F, double *__restrict__ Omean)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    double es = 0.0, oe = 0.0, o = 0.0;
    for (int s = 0; s < slices; ++s) {
        es += part_e[s];
        oe += part_oe[(int64_t)s * P + p];
        o += part_o[(int64_t)s * P + p];
    }
    const double inv = 1.0 / (double)n;
    const double om = o * inv;
    F[p] = oe * inv - om * (es * inv);
    if (Omean) Omean[p] = om;
}

nqs_status launch_forces(const float *O, const double *eloc, int64_t n, int64_t P, double *F, double *Omean,
                         hipStream_t stream)
{
    const int slices = (int)std::min<int64_t>(kForceSlices, n);
    const int64_t per = (n + slices - 1) / slices;
    const size_t need = sizeof(double) * ((size_t)2 * slices * P + slices);
    double *ws = (double *)workspace(need, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    double *poe = ws, *po = ws + (size_t)slices * P, *pe = ws + (size_t)2 * slices * P;
    const int64_t bx = (P + 255) / 256;
    if (bx > INT32_MAX) return set_error(NQS_EINVAL, "P too large");
    hipLaunchKernelGGL(forces_partial_kernel, dim3((unsigned)bx, slices), dim3(256), 0, stream, O, eloc, n, P, per, poe,
                       po, pe);
    hipLaunchKernelGGL(forces_final_kernel, dim3((unsigned)bx), dim3(256), 0, stream, poe, po, pe, slices, n, P, F, Omean);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
