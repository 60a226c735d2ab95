// Centred Gram matrices of the log-derivatives on FP32 matrix cores:
//   mode 0:  S = Obar^T Obar / n   (Eq. eq:smat, P x P)
//   mode 1:  T = Obar Obar^T / n   (n x n; same non-zero spectrum as S)
//   mode 2:  T += Obar Obar^T / n  (T summed over column blocks of O)
// with Obar = O - (column means over samples).  Centring is per column, so the
// T of a column block of O is that block's share of the whole T.
//
// Work decomposition: the output is cut into 128 x 128 tiles, of which only
// those on or above the diagonal are computed; the contraction of a tile is cut
// into steps of 32.  The grid has two blocks per compute unit.  As many whole
// rounds of tiles as the grid holds are done data-parallel (every block one
// whole tile per round, so all blocks walk the contraction together and share
// each slab of O through L2); the remaining tiles' (tile, step) pairs are laid
// end to end and every block takes one contiguous, equal share ("stream-K"), so
// no compute unit idles at the end of the launch.  A tile shared by several
// blocks is written by each of them to a per-block partial slot and summed in
// block order by a second kernel, so results do not depend on timing.  Blocks
// are renumbered so that consecutive ids land on the same XCD.
//
// Inside a block: four waves, each owns a 64 x 64 quadrant as 2 x 2
// v_mfma_f32_32x32x2f32 accumulators.  Operand tiles are staged through
// registers into double-buffered LDS (one barrier per step), centred while
// staging, and stored row-major with a 36-float row stride so that each lane
// reads its 16 contraction values with four conflict-free 128-bit loads (the
// contraction index is assigned to MFMA steps in a permuted but fixed order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "internal.h"

namespace nqs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));   // native 4-vector (no HIP wrapper struct)

constexpr int kGT = 128;                        // output tile side
constexpr int kGK = 32;                         // contraction step
constexpr int kGLd = kGK + 4;                   // LDS row stride in floats
constexpr int kGTile = kGT * kGLd;              // floats per staged operand tile
constexpr size_t kGramLds = sizeof(float) * 4 * kGTile;   // 2 buffers x (A, B): 73,728 B
constexpr int kColChunks = 64;

// ---- column means (FP64 sums over fixed row chunks, summed in chunk order) ----

__global__ void colmean_partial_kernel(const float *__restrict__ O, int64_t n, int64_t P, int chunks,
                                       double *__restrict__ part)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= P) return;
    const int64_t r0 = c * n / chunks, r1 = (c + 1) * n / chunks;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)O[r * P + p];
    part[(int64_t)c * P + p] = s;
}

__global__ void colmean_final_kernel(const double *__restrict__ part, int64_t n, int64_t P, int chunks,
                                     float *__restrict__ mu)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * P + p];
    mu[p] = (float)(s / (double)n);
}

// ---- the contraction ----

struct GramArgs {
    const float *O;     // [n][P] row-major
    const float *mu;    // [P] column means
    float *out;         // [side][side]
    float *part;        // [grid][2][kGT * kGT] partial tiles
    int64_t P;          // row length of O
    int64_t side;       // output side: n (T) or P (S)
    int64_t kdim;       // contraction length: P (T) or n (S)
    int64_t nt;         // tiles per output side
    int64_t ksteps;     // contraction steps per tile
    int64_t dp_tiles;   // tiles done whole in data-parallel rounds (a multiple of grid)
    int64_t work;       // (remaining tiles) x ksteps, shared out stream-K
    int grid;
    int accum;          // add into out instead of overwriting it
    float alpha;
};

// Block (in the renumbered order) whose share contains work item w.
__device__ __host__ inline int64_t gram_block_of(int64_t w, int64_t work, int64_t grid)
{
    return ((w + 1) * grid - 1) / work;
}

// Tile t of the upper triangle in row-major order -> (bi, bj), bi <= bj.
__device__ inline void gram_tile(int64_t t, int64_t nt, int64_t &bi, int64_t &bj)
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

// Global -> registers for contraction step ks: 4 x f32x4 of each operand per thread.
//   T: element (m, k) = O[m][k] - mu[k]; thread covers rows r + 32q, columns k4..k4+3
//   S: element (m, k) = O[k][m] - mu[m]; thread covers k-rows kk + 8q, columns m4..m4+3
template <bool TMODE, bool VEC>
__device__ inline void gram_load(const GramArgs &g, int64_t m0, int64_t ks, f32x4 (&v)[4])
{
    const int tid = threadIdx.x;
    if constexpr (TMODE) {
        const int r = tid >> 3, k4 = (tid & 7) * 4;
        const int64_t k = ks * kGK + k4;
        if constexpr (VEC) {
            const f32x4 m = k < g.kdim ? *(const f32x4 *)(g.mu + k) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = m0 + r + 32 * q;
                if (row < g.side && k < g.kdim) {
                    const f32x4 o = *(const f32x4 *)(g.O + row * g.P + k);
                    v[q] = f32x4{o.x - m.x, o.y - m.y, o.z - m.z, o.w - m.w};
                } else {
                    v[q] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = m0 + r + 32 * q;
                float e[4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    e[c] = (row < g.side && k + c < g.kdim) ? g.O[row * g.P + k + c] - g.mu[k + c] : 0.0f;
                v[q] = f32x4{e[0], e[1], e[2], e[3]};
            }
        }
    } else {
        const int kk = tid >> 5, m4 = (tid & 31) * 4;
        const int64_t m = m0 + m4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = ks * kGK + kk + 8 * q;
            if constexpr (VEC) {
                if (m < g.side && k < g.kdim) {
                    const f32x4 o = *(const f32x4 *)(g.O + k * g.P + m);
                    const f32x4 mm = *(const f32x4 *)(g.mu + m);
                    v[q] = f32x4{o.x - mm.x, o.y - mm.y, o.z - mm.z, o.w - mm.w};
                } else {
                    v[q] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            } else {
                float e[4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    e[c] = (m + c < g.side && k < g.kdim) ? g.O[k * g.P + m + c] - g.mu[m + c] : 0.0f;
                v[q] = f32x4{e[0], e[1], e[2], e[3]};
            }
        }
    }
}

// Registers -> LDS tile [kGT rows (output index)][kGLd] (contraction index contiguous).
template <bool TMODE>
__device__ inline void gram_store(float *__restrict__ dst, const f32x4 (&v)[4])
{
    const int tid = threadIdx.x;
    if constexpr (TMODE) {
        const int r = tid >> 3, k4 = (tid & 7) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) *(f32x4 *)(dst + (r + 32 * q) * kGLd + k4) = v[q];
    } else {
        const int kk = tid >> 5, m4 = (tid & 31) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dst[(m4 + 0) * kGLd + kk + 8 * q] = v[q].x;
            dst[(m4 + 1) * kGLd + kk + 8 * q] = v[q].y;
            dst[(m4 + 2) * kGLd + kk + 8 * q] = v[q].z;
            dst[(m4 + 3) * kGLd + kk + 8 * q] = v[q].w;
        }
    }
}

template <bool TMODE, bool VEC>
__global__ void __launch_bounds__(256, 2) gram_kernel(GramArgs g)
{
    extern __shared__ __align__(16) float gsm[];
    // renumber: the hardware deals blocks to the 8 XCDs round-robin
    const int x = blockIdx.x, q8 = g.grid >> 3, r8 = g.grid & 7, xcd = x & 7;
    const int lb = xcd * q8 + min(xcd, r8) + (x >> 3);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int h = lane >> 5, l32 = lane & 31;

    // contraction steps [kb, ke) of one tile; whole tiles are written out, parts go to a slot
    auto run = [&](int64_t tile, int64_t kb, int64_t ke, bool whole, int slot) {
        int64_t bi, bj;
        gram_tile(tile, g.nt, bi, bj);
        const int64_t m0 = bi * kGT, n0 = bj * kGT;

        floatx16 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

        f32x4 va[4], vb[4];
        gram_load<TMODE, VEC>(g, m0, kb, va);
        gram_load<TMODE, VEC>(g, n0, kb, vb);
        gram_store<TMODE>(gsm, va);
        gram_store<TMODE>(gsm + kGTile, vb);
        __syncthreads();
        for (int64_t ks = kb; ks < ke; ++ks) {
            const int cur = (int)((ks - kb) & 1);
            const float *As = gsm + (2 * cur) * kGTile;
            const float *Bs = As + kGTile;
            const bool more = ks + 1 < ke;
            if (more) {
                gram_load<TMODE, VEC>(g, m0, ks + 1, va);
                gram_load<TMODE, VEC>(g, n0, ks + 1, vb);
            }
#pragma unroll 1
            for (int c = 0; c < 4; ++c) {
                const int kof = h * 16 + 4 * c;
                const f32x4 a0 = *(const f32x4 *)(As + (wm + l32) * kGLd + kof);
                const f32x4 a1 = *(const f32x4 *)(As + (wm + 32 + l32) * kGLd + kof);
                const f32x4 b0 = *(const f32x4 *)(Bs + (wn + l32) * kGLd + kof);
                const f32x4 b1 = *(const f32x4 *)(Bs + (wn + 32 + l32) * kGLd + kof);
                const float av0[4] = {a0.x, a0.y, a0.z, a0.w}, av1[4] = {a1.x, a1.y, a1.z, a1.w};
                const float bv0[4] = {b0.x, b0.y, b0.z, b0.w}, bv1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0[e], bv0[e], acc[0][0], 0, 0, 0);
                    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0[e], bv1[e], acc[0][1], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1[e], bv0[e], acc[1][0], 0, 0, 0);
                    acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1[e], bv1[e], acc[1][1], 0, 0, 0);
                }
            }
            if (more) {
                float *nxt = gsm + (2 * (cur ^ 1)) * kGTile;
                gram_store<TMODE>(nxt, va);
                gram_store<TMODE>(nxt + kGTile, vb);
            }
            __syncthreads();
        }

        float *pt = g.part + ((int64_t)lb * 2 + slot) * (kGT * kGT);
        // D[i][j] of a 32x32 accumulator: lane = j + 32*((i/4)%2), register = i%4 + 4*(i/8)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ti = wm + 32 * a + 8 * (r >> 2) + 4 * h + (r & 3);
                    const int tj = wn + 32 * b + l32;
                    if (whole) {
                        const int64_t gi = m0 + ti, gj = n0 + tj;
                        if (gi < g.side && gj < g.side) {
                            const float v = g.alpha * acc[a][b][r];
                            float *o1 = g.out + gi * g.side + gj;
                            *o1 = g.accum ? *o1 + v : v;
                            if (bi != bj) {
                                float *o2 = g.out + gj * g.side + gi;
                                *o2 = g.accum ? *o2 + v : v;
                            }
                        }
                    } else {
                        pt[ti * kGT + tj] = acc[a][b][r];
                    }
                }
    };

    // data-parallel rounds: every block takes whole tiles, so all blocks walk the
    // contraction together and share each slab of O through L2
    for (int64_t t = lb; t < g.dp_tiles; t += g.grid) run(t, 0, g.ksteps, true, 0);
    // stream-K over the remaining tiles
    if (g.work > 0) {
        const int64_t w0 = (int64_t)lb * g.work / g.grid, w1 = (int64_t)(lb + 1) * g.work / g.grid;
        for (int64_t w = w0; w < w1;) {
            const int64_t kb = w % g.ksteps;
            const int64_t ke = min(g.ksteps, kb + (w1 - w));
            run(g.dp_tiles + w / g.ksteps, kb, ke, kb == 0 && ke == g.ksteps, w == w0 ? 0 : 1);
            w += ke - kb;
        }
    }
}

// Tiles shared by several blocks: sum the partial slots in block order, scale,
// and write the tile and its mirror (the mirror through an LDS transpose).
__global__ void __launch_bounds__(256) gram_fixup_kernel(GramArgs g)
{
    constexpr int kHalf = kGT / 2;
    __shared__ float tileS[kHalf][kGT + 1];
    const int64_t tile = g.dp_tiles + blockIdx.x;
    const int64_t ws = (int64_t)blockIdx.x * g.ksteps, we = ws + g.ksteps - 1;
    const int64_t blo = gram_block_of(ws, g.work, g.grid), bhi = gram_block_of(we, g.work, g.grid);
    if (blo == bhi) return;   // written whole by one block
    int64_t bi, bj;
    gram_tile(tile, g.nt, bi, bj);
    const int64_t m0 = bi * kGT, n0 = bj * kGT;
    for (int r0 = 0; r0 < kGT; r0 += kHalf) {
        for (int idx = threadIdx.x; idx < kHalf * kGT; idx += blockDim.x) {
            const int ti = r0 + idx / kGT, tj = idx % kGT;
            float s = 0.0f;
            for (int64_t b = blo; b <= bhi; ++b) {
                const int64_t wb = b * g.work / g.grid;   // first item of block b
                if (wb == (b + 1) * g.work / g.grid) continue;   // empty share
                const int slot = wb >= ws ? 0 : 1;        // b starts inside this tile, or runs into it
                s += g.part[(b * 2 + slot) * (kGT * kGT) + ti * kGT + tj];
            }
            tileS[idx / kGT][tj] = g.alpha * s;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < kHalf * kGT; idx += blockDim.x) {
            const int ti = idx / kGT, tj = idx % kGT;
            const int64_t gi = m0 + r0 + ti, gj = n0 + tj;
            if (gi < g.side && gj < g.side) {
                float *o = g.out + gi * g.side + gj;
                *o = g.accum ? *o + tileS[ti][tj] : tileS[ti][tj];
            }
        }
        if (bi != bj) {
            for (int idx = threadIdx.x; idx < kHalf * kGT; idx += blockDim.x) {
                const int tj = idx / kHalf, ti = idx % kHalf;   // mirror row n0 + tj, column m0 + r0 + ti
                const int64_t gj = n0 + tj, gi = m0 + r0 + ti;
                if (gi < g.side && gj < g.side) {
                    float *o = g.out + gj * g.side + gi;
                    *o = g.accum ? *o + tileS[ti][tj] : tileS[ti][tj];
                }
            }
        }
        __syncthreads();
    }
}

template <bool TMODE, bool VEC>
static void launch_gram_kernel(const GramArgs &g, hipStream_t stream)
{
    allow_lds(gram_kernel<TMODE, VEC>, kGramLds);
    hipLaunchKernelGGL((gram_kernel<TMODE, VEC>), dim3(g.grid), dim3(256), kGramLds, stream, g);
}

// Launch geometry shared by the workspace size and the launch.
static nqs_status gram_plan(int64_t n, int64_t P, int mode, GramArgs &g, int64_t &tiles)
{
    const bool tmode = mode != 0;
    g.P = P;
    g.side = tmode ? n : P;
    g.kdim = tmode ? P : n;
    g.nt = (g.side + kGT - 1) / kGT;
    g.ksteps = (g.kdim + kGK - 1) / kGK;
    tiles = g.nt * (g.nt + 1) / 2;
    if (tiles > INT32_MAX || tiles > INT64_MAX / g.ksteps) return set_error(NQS_EINVAL, "Gram matrix too large");
    const int64_t slots = (int64_t)device_cus() * 2;
    g.grid = (int)std::min<int64_t>(slots, tiles * g.ksteps);
    g.dp_tiles = tiles >= g.grid ? tiles / g.grid * g.grid : 0;
    g.work = (tiles - g.dp_tiles) * g.ksteps;
    g.accum = mode == 2;
    g.alpha = (float)(1.0 / (double)n);
    return NQS_OK;
}

static size_t gram_mu_bytes(int64_t P) { return (sizeof(float) * (size_t)P + 255) & ~(size_t)255; }

size_t gram_workspace_bytes(int64_t n, int64_t P)
{
    // the larger of the two modes' partial-tile areas (both use the same grid bound)
    const size_t part_bytes = sizeof(float) * (size_t)device_cus() * 2 * 2 * kGT * kGT;
    const size_t cm_bytes = sizeof(double) * (size_t)kColChunks * (size_t)P;
    (void)n;
    return gram_mu_bytes(P) + std::max(part_bytes, cm_bytes);
}

nqs_status launch_gram(const float *O, int64_t n, int64_t P, int mode, float *out, hipStream_t stream)
{
    void *ws = workspace(gram_workspace_bytes(n, P), stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    return launch_gram_ws(O, n, P, mode, out, ws, stream);
}

nqs_status launch_gram_ws(const float *O, int64_t n, int64_t P, int mode, float *out, void *wsp, hipStream_t stream)
{
    const bool tmode = mode != 0;
    GramArgs g;
    int64_t tiles = 0;
    nqs_status st = gram_plan(n, P, mode, g, tiles);
    if (st != NQS_OK) return st;
    g.O = O;
    g.out = out;
    char *ws = (char *)wsp;
    const size_t mu_bytes = gram_mu_bytes(P);
    float *mu = (float *)ws;
    g.mu = mu;
    g.part = (float *)(ws + mu_bytes);

    // column means; the partial sums reuse the space of the partial tiles
    const int chunks = (int)std::min<int64_t>(kColChunks, n);
    double *cm = (double *)(ws + mu_bytes);
    const unsigned pb = (unsigned)((P + 255) / 256);
    hipLaunchKernelGGL(colmean_partial_kernel, dim3(pb, chunks), dim3(256), 0, stream, O, n, P, chunks, cm);
    hipLaunchKernelGGL(colmean_final_kernel, dim3(pb), dim3(256), 0, stream, cm, n, P, chunks, mu);

    const bool vec = (P % 4 == 0) && ((uintptr_t)O % 16 == 0);
    if (tmode) {
        if (vec) launch_gram_kernel<true, true>(g, stream);
        else launch_gram_kernel<true, false>(g, stream);
    } else {
        if (vec) launch_gram_kernel<false, true>(g, stream);
        else launch_gram_kernel<false, false>(g, stream);
    }
    NQS_HIP_TRY(hipGetLastError());
    if (g.work > 0) {
        hipLaunchKernelGGL(gram_fixup_kernel, dim3((unsigned)(tiles - g.dp_tiles)), dim3(256), 0, stream, g);
        NQS_HIP_TRY(hipGetLastError());
    }
    return NQS_OK;
}

}  // namespace nqs
