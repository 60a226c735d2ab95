// Device helpers shared by the libnqs kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nqs {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// multiply-xor S-box; the key advances by the two Weyl constants after every
// round.  The multiplies split into mul_lo / mul_hi halves on the VALU.
// ---------------------------------------------------------------------------
struct Block4 {
    uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = c0 * 0xD2511F53u, hi0 = __umulhi(c0, 0xD2511F53u);
        const uint32_t lo1 = c2 * 0xCD9E8D57u, hi1 = __umulhi(c2, 0xCD9E8D57u);
        const uint32_t x0 = hi1 ^ c1 ^ k0;
        const uint32_t x2 = hi0 ^ c3 ^ k1;
        c0 = x0;
        c1 = lo1;
        c2 = x2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

// Stream layout: key = seed, counter = (step lo, step hi, chain, instance << 8 | tag).
__device__ __forceinline__ Block4 stream_block(uint64_t seed, uint64_t step, uint32_t chain, uint32_t inst,
                                               uint32_t tag)
{
    return philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), chain, (inst << 8) | tag, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

// floor(r * n / 2^32)
__device__ __forceinline__ int index_from_word(uint32_t r, int n)
{
    return (int)__umulhi(r, (uint32_t)n);
}

// ---------------------------------------------------------------------------
// Round an FP64 value to a format with p significand bits (implicit bit
// included) and minimum normal exponent emin: round-to-nearest-even of the
// 53-bit significand in one step, done on the integer bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double round_fp64_to_format(double x, int p, int emin, double maxfinite,
                                                        bool inf_on_overflow)
{
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    const uint64_t sign = bits >> 63;
    const int bexp = (int)((bits >> 52) & 0x7FF);
    if (bexp == 0x7FF) return x;                 // inf / nan pass through
    if (bexp == 0) return sign ? -0.0 : 0.0;     // FP64 subnormals are far below every target's range
    const int E = bexp - 1023;
    const uint64_t sig = (1ull << 52) | (bits & ((1ull << 52) - 1));
    int drop = 53 - p;
    if (E < emin) drop += emin - E;
    if (drop > 60) return sign ? -0.0 : 0.0;
    uint64_t q = sig >> drop;
    const uint64_t rem = sig & ((1ull << drop) - 1);
    const uint64_t half = 1ull << (drop - 1);
    if (rem > half || (rem == half && (q & 1ull))) q += 1;
    double r = ldexp((double)q, E - 52 + drop);
    if (r > maxfinite) r = inf_on_overflow ? __longlong_as_double(0x7FF0000000000000ll) : __longlong_as_double(0x7FF8000000000000ll);
    return sign ? -r : r;
}

// dtype codes of the public interface
enum : int { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3, kE4M3 = 4 };

__device__ __forceinline__ double round_to_dtype(double x, int dtype)
{
    switch (dtype) {
    case kF32: return round_fp64_to_format(x, 24, -126, 3.4028234663852886e38, true);
    case kF16: return round_fp64_to_format(x, 11, -14, 65504.0, true);
    case kBF16: return round_fp64_to_format(x, 8, -126, 3.3895313892515355e38, true);
    case kE4M3: return round_fp64_to_format(x, 4, -6, 448.0, false);
    default: return x;
    }
}

// ---------------------------------------------------------------------------
// Reductions inside a group of G consecutive lanes (G a power of two <= 64).
// The butterfly gives every lane of the group the bit-identical result.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int G>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// DPP reductions (no LDS traffic).  An inclusive Hillis-Steele scan inside
// each 16-lane row (row_shr 1, 2, 4, 8), then row_bcast:15 / row_bcast:31
// carry row totals upwards: the total of a group of G lanes ends in the
// group's last lane.  group_sum_uniform() hands that lane's value to the whole
// group (row_newbcast for one row, else v_readlane), so every lane of the group
// receives the same bits (decisions stay uniform).
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, false));
}

template <int G>
__device__ __forceinline__ float group_scan_total(float v)
{
    v += dpp_f32<0x111, 0xF, 0xF>(v);   // row_shr:1
    v += dpp_f32<0x112, 0xF, 0xF>(v);   // row_shr:2
    v += dpp_f32<0x114, 0xF, 0xF>(v);   // row_shr:4
    v += dpp_f32<0x118, 0xF, 0xF>(v);   // row_shr:8
    if constexpr (G >= 32) v += dpp_f32<0x142, 0xA, 0xF>(v);   // row_bcast:15 -> rows 1, 3
    if constexpr (G >= 64) v += dpp_f32<0x143, 0xC, 0xF>(v);   // row_bcast:31 -> rows 2, 3
    return v;
}

__device__ __forceinline__ float readlane_f32(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <int G>
__device__ __forceinline__ float group_sum_uniform(float v)
{
    v = group_scan_total<G>(v);
    if constexpr (G == 16) {
        return dpp_f32<0x15F, 0xF, 0xF>(v);   // row_newbcast:15: every lane of the row takes lane 15's total
    } else if constexpr (G == 64) {
        return readlane_f32(v, 63);
    } else {
        const int grp = (int)(threadIdx.x & 63) / G;
        float r = readlane_f32(v, G - 1);
#pragma unroll
        for (int q = 1; q < 64 / G; ++q) {
            const float rq = readlane_f32(v, q * G + G - 1);
            r = grp == q ? rq : r;
        }
        return r;
    }
}

// value of lane (group base + p) broadcast to the group; p is uniform
template <int G>
__device__ __forceinline__ uint32_t group_bcast(uint32_t v, int p)
{
    if constexpr (G == 64) {
        return (uint32_t)__builtin_amdgcn_readlane((int)v, p);
    } else {
        const int base = (int)(threadIdx.x & 63) & ~(G - 1);
        return (uint32_t)__shfl((int)v, base + p, 64);
    }
}

// log cosh z = |z| + log(1 + exp(-2|z|)) - log 2, FP32
__device__ __forceinline__ float logcosh_f32(float z)
{
    const float a = fabsf(z);
    return a + log1pf(__expf(-2.0f * a)) - 0.69314718055994531f;
}

}  // namespace nqs
