// Dense networks of any depth: every Metropolis step evaluates the proposed
// configurations of all chains as one batch of GEMMs on the matrix cores
// (the batched forward pass of Sec. III, one matrix product per layer).
//
// Per step (move k):
//   propose   one thread per chain draws (i, j, u) from its Philox stream; the
//             proposals that change the state (every flip, an exchange of
//             unequal spins) get a row in a compact list (atomic counter; the
//             row order does not affect any value, only where it is stored).
//   layer 1   GEMM whose A operand is built while staging: chain spins as
//             +-1 with sites i, j negated (exact in every format).
//   layer l   GEMM  H_l = ReLU(H_{l-1} W_l^T + b_l), rounded to the operand
//             format by the epilogue (the next product's input).
//   last      GEMM with a log-cosh epilogue: per row, the partial sums over
//             each 64-output slice are written, then added in slice order.
//   decide    one thread per row: Delta = 2 (f' - f) in FP32, accept iff
//             log2 u < Delta / ln 2; accepted rows flip the chain's spins and
//             keep f'.  No incremental state: f is always a full forward.
// The GEMM: 128 x 128 output tile per block of 4 waves (2 x 2 v_mfma 32x32
// tiles each), contraction steps of 128 bytes per row, operands staged
// through registers into double-buffered LDS (one barrier per step).
// Local energies use the same GEMMs on the rows (sample, connected
// configuration) of a batch of samples.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "common.h"
#include "ffnn_mc.h"
#include "internal.h"

namespace nqs {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16 staged bytes
typedef int i32x8 __attribute__((ext_vector_type(8)));             // 32 FP8 codes

// An OCP E4M3 code (1 sign, 4 exponent bits with bias 7, 3 mantissa bits) as a
// matrix-core operand.  Products on v_mfma_f32_32x32x64_f8f6f4 (both operands
// E4M3, unscaled), FP32 accumulation; a lane holds 32 consecutive K values.
struct Fp8 {
    uint8_t v;
};

template <>
struct Mc<Fp8> {
    static constexpr int EPL = 32;   // K elements per lane per instruction (K = 64)
    typedef i32x8 frag;
    static __device__ __forceinline__ mc_floatx16 mma(frag a, frag b, mc_floatx16 c)
    {
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
    }
};

// E4M3 code of v, 0 <= v < 464 (the scaled layer outputs never exceed 448), rounded to nearest even:
// normal values drop 20 of FP32's 23 mantissa bits (the carry of a round-up moves into the exponent),
// values below 2^-6 are multiples of the subnormal step 2^-9.
__device__ __forceinline__ uint32_t e4m3_code_nonneg(float v)
{
    const uint32_t x = __float_as_uint(v);
    const uint32_t nrm = ((x + 0x7FFFFu + ((x >> 20) & 1u)) >> 20) - (120u << 3);
    const uint32_t sub = (uint32_t)__builtin_rintf(v * 512.0f);
    return v < 0.015625f ? sub : nrm;
}

constexpr int kDT = 128;   // output tile side
constexpr int kDBytes = 128;   // contraction bytes per row per step

struct DeepGemmArgs {
    const void *A;             // activations [rows][lda] (operand format), when not from spins
    int lda;
    const int8_t *spins;       // [chains][N], when the A operand comes from spins
    const int *row_chain;      // row -> chain (or sample)
    const int *row_i;          // flipped sites of the row (-1: none)
    const int *row_j;
    int N;
    const int *nrows;          // device: number of rows
    const void *W;             // [Np][Kp] operand format
    const float *bias;         // [Np]
    int Kp, Nout, Np;
    void *out;                 // ReLU: [rows][ldo] operand format; log-cosh: float [rows][2 nct]
    int ldo;
    int nct;                   // output column tiles
    int max_row_tiles;
    float acc_scale;           // E4M3: accumulator -> pre-activation scale (weight scale x input scale)
    float next_inv;            // E4M3: 1 / scale of the next layer's input
};

// Bit pattern of +-1 (or 0) in the operand format.
template <typename T>
__device__ __forceinline__ uint32_t deep_pm1_bits(int s)
{
    constexpr uint32_t one = sizeof(T) == 4 ? 0x3F800000u
                           : (sizeof(T) == 1 ? 0x38u : (std::is_same<T, _Float16>::value ? 0x3C00u : 0x3F80u));
    constexpr uint32_t sign = sizeof(T) == 4 ? 0x80000000u : (sizeof(T) == 1 ? 0x80u : 0x8000u);
    return s == 0 ? 0u : (one | (s < 0 ? sign : 0u));
}

// Four 16-byte staging registers of a thread (rows r, r+32, r+64, r+96).
struct Stage4 {
    u32x4 x0, x1, x2, x3;
};

// Weights -> registers: 4 rows x 16 bytes per thread (padded, always in range).
template <typename T>
__device__ __forceinline__ void deep_load_w(const DeepGemmArgs &g, int r0, int ks, Stage4 &v)
{
    constexpr int EPC = 16 / sizeof(T), BK = kDBytes / sizeof(T);
    const int tid = threadIdx.x;
    const int k0 = ks * BK + (tid & 7) * EPC;
    const u32x4 *W = reinterpret_cast<const u32x4 *>(reinterpret_cast<const T *>(g.W) + (size_t)(r0 + (tid >> 3)) * g.Kp + k0);
    const size_t step = (size_t)32 * g.Kp * sizeof(T) / 16;
    v.x0 = W[0];
    v.x1 = W[step];
    v.x2 = W[2 * step];
    v.x3 = W[3 * step];
}

// The A operand of a GEMM: activations (AM_ACT), or the chain's spins with the row's sites negated, read 8
// (16-bit formats) or 16 (E4M3) at a time when N is a multiple of that (AM_SPINS_VEC), else one by one
// (AM_SPINS).  The AM_ACT and AM_SPINS_VEC paths have no branch: rows past the count and steps past N read a
// valid address and are zeroed by selects, so the compiler can track the loads in flight exactly (a branch
// around a load makes it wait for every outstanding load at the join).
constexpr int AM_ACT = 0, AM_SPINS_VEC = 1, AM_SPINS = 2;

// Rows -> registers (rows r0 + tid / 8 + 32 q, 16 bytes of step ks each)
template <typename T, int AM>
__device__ __forceinline__ void deep_load_a(const DeepGemmArgs &g, int r0, int ks, int nrows, const int (&rc)[4],
                                            const int (&ri)[4], const int (&rj)[4], Stage4 &v)
{
    constexpr int EPC = 16 / sizeof(T), BK = kDBytes / sizeof(T);
    const int tid = threadIdx.x;
    const int k0 = ks * BK + (tid & 7) * EPC;
    auto one = [&](int q) -> u32x4 {
        const int row = r0 + (tid >> 3) + 32 * q;
        if constexpr (AM == AM_ACT) {
            const T *A = reinterpret_cast<const T *>(g.A);
            const u32x4 d = *reinterpret_cast<const u32x4 *>(A + (size_t)(row < nrows ? row : 0) * g.lda + k0);
            const bool ok = row < nrows;
            return u32x4{ok ? d.x : 0u, ok ? d.y : 0u, ok ? d.z : 0u, ok ? d.w : 0u};
        } else if constexpr (AM == AM_SPINS_VEC) {
            static_assert(sizeof(T) <= 2, "vector spin loads for 16-bit and E4M3 operands");
            const bool ok = row < nrows && k0 < g.N;   // N is a multiple of EPC: a group is whole or past N
            const size_t at = (size_t)rc[q] * g.N + (k0 < g.N ? k0 : 0);
            uint32_t w0, w1, w2, w3;
            if constexpr (sizeof(T) == 2) {
                // 8 spins in one 8-byte load: the sign bit of each int8 (+1 = 0x01, -1 = 0xff)
                // becomes the sign bit of a 16-bit +-1; then the row's sites are negated
                const uint2 raw = *reinterpret_cast<const uint2 *>(g.spins + at);
                constexpr uint32_t one2 = std::is_same<T, _Float16>::value ? 0x3C003C00u : 0x3F803F80u;
                const uint32_t lo = (raw.x >> 7) & 0x01010101u, hi = (raw.y >> 7) & 0x01010101u;
                w0 = one2 | ((lo & 0x1u) << 15) | ((lo & 0x100u) << 23);
                w1 = one2 | ((lo & 0x10000u) >> 1) | ((lo & 0x1000000u) << 7);
                w2 = one2 | ((hi & 0x1u) << 15) | ((hi & 0x100u) << 23);
                w3 = one2 | ((hi & 0x10000u) >> 1) | ((hi & 0x1000000u) << 7);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const uint32_t e = (uint32_t)((t == 0 ? ri[q] : rj[q]) - k0);
                    const uint32_t m = e < 8u ? 1u << (15 + 16 * (e & 1u)) : 0u;
                    const uint32_t wsel = e >> 1;
                    w0 ^= wsel == 0 ? m : 0u;
                    w1 ^= wsel == 1 ? m : 0u;
                    w2 ^= wsel == 2 ? m : 0u;
                    w3 ^= wsel == 3 ? m : 0u;
                }
            } else {
                // 16 spins in one 16-byte load: +1 = 0x01, -1 = 0xff, so the E4M3 code of the spin is
                // 0x38 (1.0) with the spin's sign bit; then the row's sites are negated
                const u32x4 raw = *reinterpret_cast<const u32x4 *>(g.spins + at);
                w0 = 0x38383838u | (raw.x & 0x80808080u);
                w1 = 0x38383838u | (raw.y & 0x80808080u);
                w2 = 0x38383838u | (raw.z & 0x80808080u);
                w3 = 0x38383838u | (raw.w & 0x80808080u);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const uint32_t e = (uint32_t)((t == 0 ? ri[q] : rj[q]) - k0);
                    const uint32_t m = e < 16u ? 0x80u << (8 * (e & 3u)) : 0u;
                    const uint32_t wsel = e >> 2;
                    w0 ^= wsel == 0 ? m : 0u;
                    w1 ^= wsel == 1 ? m : 0u;
                    w2 ^= wsel == 2 ? m : 0u;
                    w3 ^= wsel == 3 ? m : 0u;
                }
            }
            return u32x4{ok ? w0 : 0u, ok ? w1 : 0u, ok ? w2 : 0u, ok ? w3 : 0u};
        } else {
            uint32_t w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
            if (row < nrows) {
                const int8_t *sp = g.spins + (size_t)rc[q] * g.N;
#pragma unroll
                for (int x = 0; x < EPC; ++x) {
                    const int k = k0 + x;
                    int sv = k < g.N ? (int)sp[k] : 0;
                    if (k == ri[q] || k == rj[q]) sv = -sv;
                    const uint32_t bits = deep_pm1_bits<T>(sv);
                    const int word = sizeof(T) == 4 ? x : (sizeof(T) == 2 ? (x >> 1) : (x >> 2));
                    const uint32_t sh = sizeof(T) == 4 ? 0u : (sizeof(T) == 2 ? 16u * (x & 1) : 8u * (x & 3));
                    if (word == 0) w0 |= bits << sh;
                    else if (word == 1) w1 |= bits << sh;
                    else if (word == 2) w2 |= bits << sh;
                    else w3 |= bits << sh;
                }
            }
            return u32x4{w0, w1, w2, w3};
        }
    };
    v.x0 = one(0);
    v.x1 = one(1);
    v.x2 = one(2);
    v.x3 = one(3);
}

template <typename T>
__device__ __forceinline__ void deep_store(T *dst, const Stage4 &v)
{
    constexpr int LD = kDBytes / sizeof(T) + 16 / sizeof(T);
    constexpr int EPC = 16 / sizeof(T);
    const int tid = threadIdx.x, c = tid & 7;
    u32x4 *p = reinterpret_cast<u32x4 *>(dst + (tid >> 3) * LD + c * EPC);
    constexpr int step = 32 * LD * sizeof(T) / 16;
    p[0] = v.x0;
    p[step] = v.x1;
    p[2 * step] = v.x2;
    p[3 * step] = v.x3;
}

// A fragment of LDS (rows are 16-byte aligned; the 32-byte FP8 fragment is read as two halves)
template <typename T>
__device__ __forceinline__ typename Mc<T>::frag deep_frag(const T *p)
{
    if constexpr (sizeof(T) == 1) {
        const u32x4 lo = *reinterpret_cast<const u32x4 *>(p), hi = *reinterpret_cast<const u32x4 *>(p + 16);
        return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    } else {
        return *reinterpret_cast<const typename Mc<T>::frag *>(p);
    }
}

template <typename T, int AM, bool LOGCOSH>
__global__ void __launch_bounds__(256, 2) deep_gemm_kernel(DeepGemmArgs g)
{
    constexpr bool SPINS = AM != AM_ACT;
    typedef typename Mc<T>::frag frag;
    constexpr int BK = kDBytes / sizeof(T);
    constexpr int LD = BK + 16 / sizeof(T);
    constexpr int EPL = Mc<T>::EPL;
    constexpr int KI = BK / (2 * EPL);            // MFMA steps per contraction step
    constexpr int TILE = kDT * LD;
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);

    const int nrows = *g.nrows;
    // The grid covers the largest row count; only `valid` tiles have work.  Block b takes tiles b, b + G,
    // b + 2G, ... (G = gridDim.x, a multiple of 8): the loads of a tile's first two contraction steps are
    // issued during the previous tile's last two, so a tile starts without waiting for memory.  Tile ids are
    // renumbered so that each XCD (blocks are dealt to the 8 XCDs round-robin) gets a contiguous range:
    // consecutive ids share a row tile, whose rows then stay in that XCD's L2.
    const int valid = ((nrows + kDT - 1) / kDT) * g.nct;
    if ((int)blockIdx.x >= valid) return;
    const int q8 = valid >> 3, r8 = valid & 7, G = gridDim.x;
    auto coords = [&](int x, int &m0, int &n0, int &ct) {
        const int xcd = x & 7, lb = xcd * q8 + min(xcd, r8) + (x >> 3);
        const int rt = lb / g.nct;
        ct = lb - rt * g.nct;
        m0 = rt * kDT;
        n0 = ct * kDT;
    };

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int l32 = lane & 31, h = lane >> 5;

    // the chain (or sample) and flipped sites of this thread's four staged rows of a tile
    auto rowinfo = [&](int m0, int (&rc)[4], int (&ri)[4], int (&rj)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rc[q] = 0;
            ri[q] = -1;
            rj[q] = -1;
            if constexpr (SPINS) {
                const int row = m0 + (tid >> 3) + 32 * q;
                if (row < nrows) {
                    rc[q] = g.row_chain[row];
                    ri[q] = g.row_i[row];
                    rj[q] = g.row_j[row];
                }
            }
        }
    };
    int x = blockIdx.x, m0, n0, ct, m0n = 0, n0n = 0, ctn = 0;
    int rc[4], ri[4], rj[4], rcn[4], rin[4], rjn[4];
    coords(x, m0, n0, ct);
    rowinfo(m0, rc, ri, rj);
    bool has_next = x + G < valid;
    if (has_next) {
        coords(x + G, m0n, n0n, ctn);
        rowinfo(m0n, rcn, rin, rjn);
    }

    mc_floatx16 acc[2][2];
    auto zero_acc = [&]() {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    };
    zero_acc();

    // The tile's output: ReLU rows in the operand format, or per-row log-cosh partials per 64-output slice.
    // The accumulators hold D[i = output][j = row]: lane = j + 32 ((i / 4) % 2), register = i % 4 + 4 (i / 8), so a
    // lane has row l32 of its 32-row block and outputs 8q + 4h + 0..3 (q = 0..3) of each 32-output block: four
    // consecutive outputs, stored together.  The bias of those outputs is read once, before any store.
    auto epilogue = [&](int m0, int n0, int ct) {
        float4 bq[2][4];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                bq[b][q] = *reinterpret_cast<const float4 *>(g.bias + n0 + wn + 32 * b + 8 * q + 4 * h);
        auto pre = [&](int a, int b, int q, int e) {   // the pre-activation of output 8q + 4h + e
            const float bb = e == 0 ? bq[b][q].x : (e == 1 ? bq[b][q].y : (e == 2 ? bq[b][q].z : bq[b][q].w));
            return std::is_same<T, Fp8>::value ? fmaf(acc[a][b][4 * q + e], g.acc_scale, bb) : acc[a][b][4 * q + e] + bb;
        };
        if constexpr (LOGCOSH) {
            float *part = reinterpret_cast<float *>(g.out);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                float abs_sum = 0.0f, prod = 1.0f;
                int cnt = 0;
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int col = n0 + wn + 32 * b + 8 * q + 4 * h + e;
                            if (col < g.Nout) {
                                const float v = fabsf(pre(a, b, q, e));
                                abs_sum += v;
                                prod *= 1.0f + __expf(-2.0f * v);   // 32 factors in (1, 2]
                                ++cnt;
                            }
                        }
                float sv = abs_sum + __logf(prod) - (float)cnt * kLn2f;
                sv += __shfl_xor(sv, 32, 64);
                const int row = m0 + wm + 32 * a + l32;
                if (h == 0 && row < nrows) part[(size_t)row * (2 * g.nct) + 2 * ct + (wn >> 6)] = sv;
            }
        } else {
            struct alignas(4 * sizeof(T)) Out4 {
                T v[4];
            };
            T *out = reinterpret_cast<T *>(g.out);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int row = m0 + wm + 32 * a + l32;
                if (row >= nrows) continue;
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int col0 = n0 + wn + 32 * b + 8 * q + 4 * h;
                        if (col0 >= g.ldo) continue;   // ldo is a multiple of 4: the group is whole
                        Out4 o;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float v = col0 + e < g.Nout ? fmaxf(pre(a, b, q, e), 0.0f) : 0.0f;
                            if constexpr (std::is_same<T, Fp8>::value)
                                // the next layer's input: ReLU(z) / s_next as an E4M3 code (s_next a power of two)
                                o.v[e] = Fp8{(uint8_t)e4m3_code_nonneg(v * g.next_inv)};
                            else
                                o.v[e] = Mc<T>::from_f32(v);
                        }
                        *reinterpret_cast<Out4 *>(out + (size_t)row * g.ldo + col0) = o;
                    }
            }
        }
    };

    // Contraction steps of all the block's tiles in sequence (ksteps >= 2 whenever a block has more than one
    // tile).  Two register stages: the loads of step v + 2 are issued before step v is computed, so each
    // global load has two steps of matrix-core work to land; across a tile boundary they are the next tile's.
    const int ksteps = g.Kp / BK;
    const int ntile = (valid - 1 - (int)blockIdx.x) / G + 1;
    const int V = ntile * ksteps;
    int ks = 0;   // step within the current tile
    // loads of step ks + d of the sequence (ksd = ks + d), without a branch: past the current tile they are
    // the next tile's; past the block's last step they read the current tile again and are never stored
    auto load = [&](int ksd, Stage4 &av, Stage4 &bv) {
        const bool nxt = ksd >= ksteps && has_next;
        int k = ksd >= ksteps ? ksd - ksteps : ksd;
        k = k < ksteps ? k : 0;
        int rca[4], ria[4], rja[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rca[q] = nxt ? rcn[q] : rc[q];
            ria[q] = nxt ? rin[q] : ri[q];
            rja[q] = nxt ? rjn[q] : rj[q];
        }
        deep_load_a<T, AM>(g, nxt ? m0n : m0, k, nrows, rca, ria, rja, av);
        deep_load_w<T>(g, nxt ? n0n : n0, k, bv);
    };
    Stage4 a0s, b0s, a1s, b1s;
    load(0, a0s, b0s);
    load(1, a1s, b1s);
    deep_store<T>(lds, a0s);
    deep_store<T>(lds + TILE, b0s);
    __syncthreads();
    auto step = [&](int v, Stage4 &af, Stage4 &bf, const Stage4 &an, const Stage4 &bn) {
        const int cur = v & 1;
        const T *As = lds + (2 * cur) * TILE;
        const T *Bs = As + TILE;
        load(ks + 2, af, bf);
#pragma unroll
        for (int kk = 0; kk < KI; ++kk) {
            const int ko = kk * 2 * EPL + EPL * h;
            const frag a0 = deep_frag<T>(As + (wm + l32) * LD + ko);
            const frag a1 = deep_frag<T>(As + (wm + 32 + l32) * LD + ko);
            const frag b0 = deep_frag<T>(Bs + (wn + l32) * LD + ko);
            const frag b1 = deep_frag<T>(Bs + (wn + 32 + l32) * LD + ko);
            // D[i = output][j = row]
            acc[0][0] = Mc<T>::mma(b0, a0, acc[0][0]);
            acc[0][1] = Mc<T>::mma(b1, a0, acc[0][1]);
            acc[1][0] = Mc<T>::mma(b0, a1, acc[1][0]);
            acc[1][1] = Mc<T>::mma(b1, a1, acc[1][1]);
        }
        {   // after the last step this fills a buffer nothing reads
            T *nxt = lds + (2 * (cur ^ 1)) * TILE;
            deep_store<T>(nxt, an);
            deep_store<T>(nxt + TILE, bn);
        }
        __syncthreads();
        if (++ks == ksteps) {   // the tile is complete: its output, then the next tile becomes current
            epilogue(m0, n0, ct);
            zero_acc();
            ks = 0;
            x += G;
            m0 = m0n;
            n0 = n0n;
            ct = ctn;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rc[q] = rcn[q];
                ri[q] = rin[q];
                rj[q] = rjn[q];
            }
            has_next = x + G < valid;
            if (has_next) {
                coords(x + G, m0n, n0n, ctn);
                rowinfo(m0n, rcn, rin, rjn);
            }
        }
    };
    for (int v = 0; v < V; v += 2) {
        step(v, a0s, b0s, a1s, b1s);
        if (v + 1 < V) step(v + 1, a1s, b1s, a0s, b0s);
    }
}

// ---------------------------------------------------------------------------
// Sampler steps
// ---------------------------------------------------------------------------
struct DeepStepArgs {
    int8_t *state;            // [C][N] live chain states
    int64_t C;
    int N, move;
    uint64_t seed, step_offset;
    uint32_t inst, chain_id_offset;
    int *counter;             // [2] rows of the current / next step
    int *row_chain, *row_i, *row_j;
    uint32_t *ubits;          // [C] u bits of the chain's current proposal
    float *fcur;              // [C] log|psi| of the current state
    const float *part;        // [rows][npart]
    int npart;
    unsigned long long *acc;  // [C]
    int64_t total;            // proposals per chain in this call
    const int64_t *kbase;     // device: index of the current sweep's first proposal (graph replays), or NULL
    int n_traced;
    int32_t *tr_site;
    uint32_t *tr_ubits;
    float *tr_delta;
    uint8_t *tr_acc;
};

__global__ void deep_propose_kernel(DeepStepArgs a, int64_t kk)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const int64_t k = (a.kbase ? *a.kbase : 0) + kk;
    const uint64_t step = a.step_offset + (uint64_t)k;
    const uint32_t gid = a.chain_id_offset + (uint32_t)c;
    const Block4 rb = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), gid, a.inst << 8, (uint32_t)a.seed,
                                    (uint32_t)(a.seed >> 32));
    const int i = index_from_word(rb.r0, a.N);
    int j = -1;
    if (a.move == 1) {
        j = index_from_word(rb.r1, a.N - 1);
        j += (j >= i) ? 1 : 0;
    }
    const int8_t *s = a.state + c * a.N;
    const bool eff = j < 0 || s[i] != s[j];
    // (row order depends on timing; no value does)
    const uint32_t ub = rb.r2 >> 8;
    a.ubits[c] = ub;
    if (eff) {
        const int r = atomicAdd(a.counter + (k & 1), 1);
        a.row_chain[r] = (int)c;
        a.row_i[r] = i;
        a.row_j[r] = j;
    } else {
        ++a.acc[c];   // a move that changes nothing is accepted
    }
    if (c < a.n_traced) {
        const size_t idx = (size_t)c * (size_t)a.total + (size_t)k;
        a.tr_site[idx] = i | ((j < 0 ? 0xFFFF : j) << 16);
        a.tr_ubits[idx] = ub;
        if (!eff) {
            a.tr_delta[idx] = 0.0f;
            a.tr_acc[idx] = 1;
        }
    }
}

__global__ void deep_decide_kernel(DeepStepArgs a, int64_t kk)
{
    const int64_t k = (a.kbase ? *a.kbase : 0) + kk;
    const int n = a.counter[k & 1];
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r == 0) a.counter[(k + 1) & 1] = 0;   // the next step's counter (not in use now)
    if (r >= n) return;
    const int c = a.row_chain[r];
    float fnew = 0.0f;
    for (int p = 0; p < a.npart; ++p) fnew += a.part[(size_t)r * a.npart + p];
    const float d2 = 2.0f * (fnew - a.fcur[c]) / kLn2f;
    const uint32_t ub = a.ubits[c];
    const float l2u = __builtin_amdgcn_logf((float)ub * 5.9604644775390625e-8f);
    const bool accept = l2u < d2;   // NaN rejects
    if (accept) {
        int8_t *s = a.state + (size_t)c * a.N;
        const int i = a.row_i[r], j = a.row_j[r];
        s[i] = -s[i];
        if (j >= 0) s[j] = -s[j];
        a.fcur[c] = fnew;
        ++a.acc[c];
    }
    if (c < a.n_traced) {
        const size_t idx = (size_t)c * (size_t)a.total + (size_t)k;
        a.tr_delta[idx] = d2 * kLn2f;
        a.tr_acc[idx] = accept ? 1 : 0;
    }
}

// rows = all chains, nothing flipped (the initial forward pass)
__global__ void deep_rows_all_kernel(int64_t C, int *counter, int *row_chain, int *row_i, int *row_j)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c == 0) {
        counter[0] = (int)C;
        counter[1] = 0;
    }
    if (c >= C) return;
    row_chain[c] = (int)c;
    row_i[c] = -1;
    row_j[c] = -1;
}

__global__ void deep_set_f_kernel(int64_t C, const float *part, int npart, float *fcur, int *counter,
                                  unsigned long long *acc)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c == 0) counter[0] = 0;
    if (c >= C) return;
    float f = 0.0f;
    for (int p = 0; p < npart; ++p) f += part[(size_t)c * npart + p];
    fcur[c] = f;
    acc[c] = 0ull;
}

__global__ void deep_emit_kernel(const int8_t *state, int64_t C, int N, const float *fcur, int8_t *samples,
                                 float *logpsi)
{
    const int64_t n = C * N;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        if (samples) samples[p] = state[p];
        if (logpsi && p < C) logpsi[p] = fcur[p];
    }
}

// graph replays: the emit of the sweep that starts at proposal *kbase, then the advance to the next sweep
__global__ void deep_emit_sweep_kernel(const int8_t *state, int64_t C, int N, const float *fcur, int8_t *samples,
                                       float *logpsi, const int64_t *kbase, int sweep_size, int n_burnin, int n_sweeps)
{
    const int64_t out = *kbase / sweep_size - n_burnin;
    if (out < 0 || out >= n_sweeps) return;
    const int64_t n = C * N;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        if (samples) samples[(size_t)out * n + p] = state[p];
        if (logpsi && p < C) logpsi[(size_t)out * C + p] = fcur[p];
    }
}

__global__ void deep_set_i64_kernel(int64_t *p, int64_t v, int64_t add)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = add ? *p + add : v;
}

__global__ void deep_copy_acc_kernel(const unsigned long long *acc, int64_t C, uint64_t *out)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c < C) out[c] = acc[c];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <typename T, int AM, bool LOGCOSH>
static void deep_gemm_launch(const DeepGemmArgs &g, hipStream_t s)
{
    constexpr size_t lds = 4 * sizeof(T) * kDT * (kDBytes / sizeof(T) + 16 / sizeof(T));
    allow_lds(deep_gemm_kernel<T, AM, LOGCOSH>, lds);
    // persistent blocks (two per CU, a multiple of 8 for the XCD renumbering) when a tile has at least two
    // contraction steps; otherwise one block per tile
    int blocks = g.max_row_tiles * g.nct;
    if (g.Kp / (kDBytes / (int)sizeof(T)) >= 2) blocks = std::min(blocks, 2 * device_cus());
    hipLaunchKernelGGL((deep_gemm_kernel<T, AM, LOGCOSH>), dim3(blocks), dim3(256), lds, s, g);
}

template <typename T>
static void deep_gemm_dispatch(bool spins, bool logcosh, const DeepGemmArgs &g, hipStream_t s)
{
    // spins read EPC at a time when N is a multiple of EPC (16-bit and E4M3 operands)
    constexpr int EPC = 16 / sizeof(T);
    if (spins && sizeof(T) <= 2 && g.N % EPC == 0) {
        if constexpr (sizeof(T) <= 2) {
            if (logcosh) deep_gemm_launch<T, AM_SPINS_VEC, true>(g, s);
            else deep_gemm_launch<T, AM_SPINS_VEC, false>(g, s);
        }
    } else if (spins) {
        if (logcosh) deep_gemm_launch<T, AM_SPINS, true>(g, s);
        else deep_gemm_launch<T, AM_SPINS, false>(g, s);
    } else {
        if (logcosh) deep_gemm_launch<T, AM_ACT, true>(g, s);
        else deep_gemm_launch<T, AM_ACT, false>(g, s);
    }
}

// Scratch of one forward pass over up to `cap` rows.
struct DeepBuffers {
    int *counter, *row_chain, *row_i, *row_j;
    void *H[2];
    float *part;
    int maxK, npart;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t deep_buffer_bytes(const FfnnDev &f, int64_t cap, int esize)
{
    int maxK = 64;
    for (int l = 1; l < f.n_layers; ++l) maxK = std::max(maxK, f.Kp[l]);
    const int npart = 2 * (f.Np[f.n_layers - 1] / kDT);
    return al256(sizeof(int) * 2) + 3 * al256(sizeof(int) * cap) + 2 * al256((size_t)esize * cap * maxK) +
           al256(sizeof(float) * cap * npart);
}

static DeepBuffers deep_carve(const FfnnDev &f, int64_t cap, int esize, char *base)
{
    DeepBuffers b;
    b.maxK = 64;
    for (int l = 1; l < f.n_layers; ++l) b.maxK = std::max(b.maxK, f.Kp[l]);
    b.npart = 2 * (f.Np[f.n_layers - 1] / kDT);
    auto carve = [&](size_t sz) {
        char *p = base;
        base += al256(sz);
        return p;
    };
    b.counter = (int *)carve(sizeof(int) * 2);
    b.row_chain = (int *)carve(sizeof(int) * cap);
    b.row_i = (int *)carve(sizeof(int) * cap);
    b.row_j = (int *)carve(sizeof(int) * cap);
    b.H[0] = carve((size_t)esize * cap * b.maxK);
    b.H[1] = carve((size_t)esize * cap * b.maxK);
    b.part = (float *)carve(sizeof(float) * cap * b.npart);
    return b;
}

// One forward pass of the rows listed in b (count on the device), spins from `spins`.
static void deep_forward(int dtype, const FfnnDev &f, const DeepBuffers &b, const int8_t *spins, int64_t cap,
                         hipStream_t s)
{
    const int L = f.n_layers;
    DeepGemmArgs g;
    g.spins = spins;
    g.row_chain = b.row_chain;
    g.row_i = b.row_i;
    g.row_j = b.row_j;
    g.N = f.widths[0];
    g.nrows = b.counter;
    g.max_row_tiles = (int)((cap + kDT - 1) / kDT);
    for (int l = 0; l < L; ++l) {
        const bool last = l == L - 1;
        g.A = l == 0 ? nullptr : b.H[(l - 1) & 1];
        g.lda = f.Kp[l];
        g.W = f.Wd[l];
        g.bias = f.bd[l];
        g.Kp = f.Kp[l];
        g.Nout = f.widths[l + 1];
        g.Np = f.Np[l];
        g.nct = f.Np[l] / kDT;
        g.out = last ? (void *)b.part : b.H[l & 1];
        g.ldo = last ? 0 : f.Kp[l + 1];
        g.acc_scale = f.acc_scale[l];
        g.next_inv = f.next_inv[l];
        if (dtype == NQS_F16) deep_gemm_dispatch<_Float16>(l == 0, last, g, s);
        else if (dtype == NQS_BF16) deep_gemm_dispatch<__bf16>(l == 0, last, g, s);
        else if (dtype == NQS_FP8_E4M3) deep_gemm_dispatch<Fp8>(l == 0, last, g, s);
        else deep_gemm_dispatch<float>(l == 0, last, g, s);
    }
}

nqs_status deep_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                       uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream)
{
    const FfnnDev &f = m->copies[cfg.dtype].ffnn;
    const int N = f.widths[0];
    const int64_t C = cfg.n_chains;
    const int esize = cfg.dtype == NQS_F32 ? 4 : (cfg.dtype == NQS_FP8_E4M3 ? 1 : 2);
    if (C > INT32_MAX / 2) return set_error(NQS_EINVAL, "too many chains");
    // scratch: forward buffers + per-chain state
    const size_t fwd = deep_buffer_bytes(f, C, esize);
    const size_t per_chain = al256(sizeof(uint32_t) * C) + al256(sizeof(float) * C) + al256(sizeof(unsigned long long) * C) +
                             al256(sizeof(int64_t));
    char *ws = (char *)workspace(fwd + per_chain, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    DeepBuffers b = deep_carve(f, C, esize, ws);
    char *pc = ws + fwd;
    uint32_t *ubits = (uint32_t *)pc;
    float *fcur = (float *)(pc + al256(sizeof(uint32_t) * C));
    unsigned long long *acc = (unsigned long long *)(pc + al256(sizeof(uint32_t) * C) + al256(sizeof(float) * C));
    int64_t *kbase = (int64_t *)(pc + al256(sizeof(uint32_t) * C) + al256(sizeof(float) * C) +
                                 al256(sizeof(unsigned long long) * C));

    if (cfg.init_chains) {
        nqs_status st = launch_init_chains(chain_state, C, N, cfg.move, cfg.seed, cfg.instance_id, cfg.chain_id_offset,
                                           stream);
        if (st != NQS_OK) return st;
    }
    const unsigned cb = (unsigned)((C + 255) / 256);
    // f of the start states
    hipLaunchKernelGGL(deep_rows_all_kernel, dim3(cb), dim3(256), 0, stream, C, b.counter, b.row_chain, b.row_i, b.row_j);
    deep_forward(cfg.dtype, f, b, chain_state, C, stream);
    hipLaunchKernelGGL(deep_set_f_kernel, dim3(cb), dim3(256), 0, stream, C, b.part, b.npart, fcur, b.counter, acc);
    NQS_HIP_TRY(hipGetLastError());

    DeepStepArgs a;
    a.state = chain_state;
    a.C = C;
    a.N = N;
    a.move = cfg.move;
    a.seed = cfg.seed;
    a.step_offset = cfg.step_offset;
    a.inst = cfg.instance_id;
    a.chain_id_offset = (uint32_t)cfg.chain_id_offset;
    a.counter = b.counter;
    a.row_chain = b.row_chain;
    a.row_i = b.row_i;
    a.row_j = b.row_j;
    a.ubits = ubits;
    a.fcur = fcur;
    a.part = b.part;
    a.npart = b.npart;
    a.acc = acc;
    const int sw = cfg.sweep_size > 0 ? cfg.sweep_size : N;
    a.total = (int64_t)(cfg.n_burnin + cfg.n_sweeps) * sw;
    const bool tr = trace && trace->n_chains_traced > 0;
    a.n_traced = tr ? trace->n_chains_traced : 0;
    a.tr_site = tr ? trace->site : nullptr;
    a.tr_ubits = tr ? trace->ubits : nullptr;
    a.tr_delta = tr ? trace->delta : nullptr;
    a.tr_acc = tr ? trace->accepted : nullptr;
    a.kbase = nullptr;

    // Two or more sweeps of an even size: capture one sweep's launches (proposal, forward pass, decision for each
    // of its proposals, then the sample emit) once into a graph and replay it per sweep; the proposal index and
    // the sweep come from a device counter that the graph's last node advances, so every replay is the same graph.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    NQS_HIP_TRY(hipStreamIsCapturing(stream, &cap));
    const int n_sw = cfg.n_burnin + cfg.n_sweeps;
    if (sw % 2 == 0 && n_sw >= 2 && cap == hipStreamCaptureStatusNone) {
        a.kbase = kbase;
        hipLaunchKernelGGL(deep_set_i64_kernel, dim3(1), dim3(1), 0, stream, kbase, (int64_t)0, (int64_t)0);
        std::string sig;
        auto add = [&](const void *p, size_t n) { sig.append((const char *)p, n); };
        add(&a, sizeof(a));
        add(&b, sizeof(b));
        add(&f, sizeof(f));
        const int64_t ints[6] = {cfg.dtype, C, sw, cfg.n_burnin, cfg.n_sweeps, N};
        add(ints, sizeof(ints));
        add(&samples, sizeof(samples));
        add(&logpsi, sizeof(logpsi));
        if (!m->sweep_exec || m->sweep_sig != sig) {
            if (m->sweep_exec) {
                // the previous graph may still run on another stream
                if (m->sweep_done) NQS_HIP_TRY(hipEventSynchronize(m->sweep_done));
                NQS_HIP_TRY(hipGraphExecDestroy(m->sweep_exec));
                m->sweep_exec = nullptr;
            }
            hipStream_t cs = capture_stream();
            if (!cs) return set_error(NQS_EDEVICE, "could not create the capture stream");
            NQS_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
            for (int j = 0; j < sw; ++j) {
                hipLaunchKernelGGL(deep_propose_kernel, dim3(cb), dim3(256), 0, cs, a, (int64_t)j);
                DeepBuffers bk = b;
                bk.counter = b.counter + (j & 1);   // k = kbase + j with kbase even
                deep_forward(cfg.dtype, f, bk, chain_state, C, cs);
                hipLaunchKernelGGL(deep_decide_kernel, dim3(cb), dim3(256), 0, cs, a, (int64_t)j);
            }
            if (samples || logpsi) {
                const int eb = (int)std::min<int64_t>((C * N + 255) / 256, 8192);
                hipLaunchKernelGGL(deep_emit_sweep_kernel, dim3(eb), dim3(256), 0, cs, chain_state, C, N, fcur, samples,
                                   logpsi, (const int64_t *)kbase, sw, cfg.n_burnin, cfg.n_sweeps);
            }
            hipLaunchKernelGGL(deep_set_i64_kernel, dim3(1), dim3(1), 0, cs, kbase, (int64_t)0, (int64_t)sw);
            hipGraph_t graph = nullptr;
            const hipError_t e1 = hipStreamEndCapture(cs, &graph);
            if (e1 != hipSuccess || !graph) return set_error(NQS_EDEVICE, "stream capture of the sweep failed");
            const hipError_t e2 = hipGraphInstantiate(&m->sweep_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e2 != hipSuccess) {
                m->sweep_exec = nullptr;
                return set_error(NQS_EDEVICE, "graph instantiation failed");
            }
            m->sweep_sig = sig;
            if (!m->sweep_done) NQS_HIP_TRY(hipEventCreateWithFlags(&m->sweep_done, hipEventDisableTiming));
        }
        for (int q = 0; q < n_sw; ++q) NQS_HIP_TRY(hipGraphLaunch(m->sweep_exec, stream));
        NQS_HIP_TRY(hipEventRecord(m->sweep_done, stream));
        if (n_accepted) hipLaunchKernelGGL(deep_copy_acc_kernel, dim3(cb), dim3(256), 0, stream, acc, C, n_accepted);
        NQS_HIP_TRY(hipGetLastError());
        return NQS_OK;
    }

    int in_sweep = 0;
    int64_t sweep = 0;
    for (int64_t k = 0; k < a.total; ++k) {
        // rows of step k are counted in counter[k & 1]; the forward pass reads that slot
        hipLaunchKernelGGL(deep_propose_kernel, dim3(cb), dim3(256), 0, stream, a, k);
        DeepBuffers bk = b;
        bk.counter = b.counter + (k & 1);
        deep_forward(cfg.dtype, f, bk, chain_state, C, stream);
        hipLaunchKernelGGL(deep_decide_kernel, dim3(cb), dim3(256), 0, stream, a, k);
        if (++in_sweep == sw) {
            in_sweep = 0;
            const int64_t out = sweep - cfg.n_burnin;
            if (out >= 0 && (samples || logpsi)) {
                const int eb = (int)std::min<int64_t>((C * N + 255) / 256, 8192);
                hipLaunchKernelGGL(deep_emit_kernel, dim3(eb), dim3(256), 0, stream, chain_state, C, N, fcur,
                                   samples ? samples + (size_t)out * C * N : nullptr,
                                   logpsi ? logpsi + (size_t)out * C : nullptr);
            }
            ++sweep;
        }
    }
    if (n_accepted) hipLaunchKernelGGL(deep_copy_acc_kernel, dim3(cb), dim3(256), 0, stream, acc, C, n_accepted);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// ---------------------------------------------------------------------------
// Local energies: rows (sample, connected configuration), a batch at a time
// ---------------------------------------------------------------------------
struct DeepElocRowsArgs {
    const int8_t *samples;
    int64_t s0;               // first sample of the batch
    int N, kind, dim, L, pbc, marshall;
    double J, h;
    int *counter;             // rows of the batch
    int *row_chain, *row_i, *row_j;
    float *row_coef;
    int *base;                // [batch] first row of each sample (its own configuration)
    int *count;               // [batch] rows of each sample
    double *diag;             // [batch]
};

// One block (256 threads) per sample of the batch.
__global__ void __launch_bounds__(256) deep_eloc_rows_kernel(DeepElocRowsArgs a)
{
    __shared__ int s_wcount[4], s_base;
    __shared__ double s_red[4];
    const int sb = blockIdx.x;
    const int64_t smp = a.s0 + sb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int8_t *sp = a.samples + smp * a.N;
    const int nb = a.dim == 1 ? (a.pbc ? a.L : a.L - 1) : 2 * a.L * a.L;
    const int ncand = a.kind == NQS_TFIM ? a.N : 0;
    const int nloop = ncand > nb ? ncand : nb;
    // first pass: count the rows of this sample
    int mine = 0;
    double dg = 0.0;
    for (int c = tid; c < nloop; c += 256) {
        bool take = c < ncand;
        if (c < nb) {
            int bi, bj;
            bool valid = true;
            if (a.dim == 1) {
                bi = c;
                bj = c + 1 < a.L ? c + 1 : 0;
            } else {
                const int site = c >> 1, x = site / a.L, y = site % a.L;
                bi = site;
                if ((c & 1) == 0) {
                    valid = a.pbc || x + 1 < a.L;
                    bj = ((x + 1) % a.L) * a.L + y;
                } else {
                    valid = a.pbc || y + 1 < a.L;
                    bj = x * a.L + (y + 1) % a.L;
                }
            }
            if (valid) {
                dg += a.J * (double)(sp[bi] * sp[bj]);
                if (a.kind == NQS_HEISENBERG && sp[bi] != sp[bj]) take = true;
            }
        }
        mine += take ? 1 : 0;
    }
    int tot = mine;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
    if (lane == 0) s_wcount[wave] = tot;
    const double dsum = group_sum<64>(dg);
    if (lane == 0) s_red[wave] = dsum;
    __syncthreads();
    if (tid == 0) {
        const int rows = 1 + s_wcount[0] + s_wcount[1] + s_wcount[2] + s_wcount[3];
        const int b0 = atomicAdd(a.counter, rows);
        s_base = b0;
        a.base[sb] = b0;
        a.count[sb] = rows;
        a.diag[sb] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
        a.row_chain[b0] = (int)smp;
        a.row_i[b0] = -1;
        a.row_j[b0] = -1;
        a.row_coef[b0] = 0.0f;
    }
    __syncthreads();
    // second pass: write the rows in candidate order
    int pos = s_base + 1;
    for (int base = 0; base < nloop; base += 256) {
        const int c = base + tid;
        int i = -1, j = -1;
        bool take = false;
        float coef = 0.0f;
        if (c < ncand) {
            i = c;
            take = true;
            coef = (float)a.h * ((a.marshall && on_sub_a(a.dim, a.L, i)) ? -1.0f : 1.0f);
        }
        if (c < nb && a.kind == NQS_HEISENBERG) {
            int bi, bj;
            bool valid = true;
            if (a.dim == 1) {
                bi = c;
                bj = c + 1 < a.L ? c + 1 : 0;
            } else {
                const int site = c >> 1, x = site / a.L, y = site % a.L;
                bi = site;
                if ((c & 1) == 0) {
                    valid = a.pbc || x + 1 < a.L;
                    bj = ((x + 1) % a.L) * a.L + y;
                } else {
                    valid = a.pbc || y + 1 < a.L;
                    bj = x * a.L + (y + 1) % a.L;
                }
            }
            if (valid && sp[bi] != sp[bj]) {
                i = bi;
                j = bj;
                take = true;
                const bool flip = a.marshall && (on_sub_a(a.dim, a.L, bi) != on_sub_a(a.dim, a.L, bj));
                coef = 2.0f * (float)a.J * (flip ? -1.0f : 1.0f);
            }
        }
        const unsigned long long bal = __ballot(take);
        __syncthreads();
        if (lane == 0) s_wcount[wave] = __popcll(bal);
        __syncthreads();
        int off = pos;
        for (int w = 0; w < wave; ++w) off += s_wcount[w];
        if (take) {
            const int r = off + __popcll(bal & ((1ull << lane) - 1ull));
            a.row_chain[r] = (int)smp;
            a.row_i[r] = i;
            a.row_j[r] = j;
            a.row_coef[r] = coef;
        }
        pos += s_wcount[0] + s_wcount[1] + s_wcount[2] + s_wcount[3];
    }
}

// One wave per sample: eps = diag + sum_rows coef exp(f_row - f_sample) (FP64).
__global__ void deep_eloc_reduce_kernel(int nb, const int *base, const int *count, const double *diag,
                                        const float *row_coef, const float *part, int npart, double *eloc)
{
    const int sb = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (sb >= nb) return;
    const int b0 = base[sb], n = count[sb];
    auto fof = [&](int r) {
        float f = 0.0f;
        for (int p = 0; p < npart; ++p) f += part[(size_t)r * npart + p];
        return f;
    };
    const float f0 = fof(b0);
    double off = 0.0;
    for (int r = 1 + lane; r < n; r += 64) off += (double)row_coef[b0 + r] * exp((double)(fof(b0 + r) - f0));
    off = group_sum<64>(off);
    if (lane == 0) eloc[sb] = diag[sb] + off;
}

nqs_status deep_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                             double *eloc, hipStream_t stream)
{
    const FfnnDev &f = m->copies[dtype].ffnn;
    const int N = f.widths[0];
    const int esize = dtype == NQS_F32 ? 4 : (dtype == NQS_FP8_E4M3 ? 1 : 2);
    const int per = 2 * N + 1;                               // rows per sample at most
    const int64_t cap = std::max<int64_t>(per, std::min<int64_t>(65536, (int64_t)per * std::max<int64_t>(1, n)));
    const int bs = (int)std::max<int64_t>(1, cap / per);     // samples per batch
    const size_t fwd = deep_buffer_bytes(f, cap, esize);
    const size_t extra = al256(sizeof(float) * cap) + 2 * al256(sizeof(int) * bs) + al256(sizeof(double) * bs);
    char *ws = (char *)workspace(fwd + extra, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    DeepBuffers b = deep_carve(f, cap, esize, ws);
    char *pe = ws + fwd;
    float *row_coef = (float *)pe;
    int *base = (int *)(pe + al256(sizeof(float) * cap));
    int *count = (int *)(pe + al256(sizeof(float) * cap) + al256(sizeof(int) * bs));
    double *diag = (double *)(pe + al256(sizeof(float) * cap) + 2 * al256(sizeof(int) * bs));

    DeepElocRowsArgs a;
    a.samples = samples;
    a.N = N;
    a.kind = ham.kind;
    a.dim = ham.dim;
    a.L = ham.L;
    a.pbc = ham.pbc;
    a.marshall = m->desc.marshall;
    a.J = ham.J;
    a.h = ham.h;
    a.counter = b.counter;
    a.row_chain = b.row_chain;
    a.row_i = b.row_i;
    a.row_j = b.row_j;
    a.row_coef = row_coef;
    a.base = base;
    a.count = count;
    a.diag = diag;
    for (int64_t s0 = 0; s0 < n; s0 += bs) {
        const int nbat = (int)std::min<int64_t>(bs, n - s0);
        a.s0 = s0;
        nqs_status z = launch_zero_u64(b.counter, 1, stream);
        if (z != NQS_OK) return z;
        hipLaunchKernelGGL(deep_eloc_rows_kernel, dim3(nbat), dim3(256), 0, stream, a);
        deep_forward(dtype, f, b, samples, cap, stream);
        hipLaunchKernelGGL(deep_eloc_reduce_kernel, dim3((nbat + 3) / 4), dim3(256), 0, stream, nbat, base, count, diag,
                           row_coef, b.part, b.npart, eloc + s0);
        NQS_HIP_TRY(hipGetLastError());
    }
    return NQS_OK;
}

}  // namespace nqs
