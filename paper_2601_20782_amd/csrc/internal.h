// Host-side internals of libnqs: the model handle, error reporting, workspace,
// and the launch entry points each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "nqs.h"

namespace nqs {

// Thread-local message of the last failing call.
nqs_status set_error(nqs_status st, const std::string &msg);
nqs_status hip_error(hipError_t e, const char *what);

#define NQS_HIP_TRY(expr)                                   \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return ::nqs::hip_error(_e, #expr); \
    } while (0)

// Device copy of an RBM in one sampling format.  All arrays hold FP32 numbers
// that are exactly the values of the format-rounded parameters.
struct RbmDev {
    int N = 0, M = 0;
    float *a = nullptr;       // [N]
    float *a2 = nullptr;      // [N]      4 a_i / ln 2 (the visible-bias term of a flip in log2 units)
    float *b = nullptr;       // [M]
    float *Wt = nullptr;      // [N][M]   Wt[i][j] = W[j][i]
    float2 *CS = nullptr;     // [N*M+1]  (cosh 2W[j][i], sinh 2W[j][i]) at [i][j]; entry N*M = (1, 0)
    float2 *CSt = nullptr;    // [M][N]   the same pairs at [j][i], then 8 N slack entries
    float max_abs_w = 0.0f;
};

// Dense-network copy in one sampling format.
struct FfnnDev {
    int n_layers = 0;
    int widths[NQS_MAX_LAYERS + 1] = {0};  // widths[0] = N
    float *W[NQS_MAX_LAYERS] = {nullptr};  // [w_l][w_{l-1}] FP32 values of the rounded weights
    float *Wt[NQS_MAX_LAYERS] = {nullptr}; // [w_{l-1}][w_l]
    float *b[NQS_MAX_LAYERS] = {nullptr};
    // matrix-core path of a two-layer network (w1 padded to m1p, w2 to m2p)
    int m1p = 0, m2p = 0;
    uint16_t *W2c = nullptr;               // [m2p][m1p] raw bf16/f16 codes of layer 2
    uint16_t *W1ct = nullptr;              // [N][m1p]   raw codes of layer 1, transposed
    float *W2p = nullptr;                  // [m2p][m1p] FP32 values of layer 2
    float *W1tp = nullptr;                 // [N][m1p]   FP32 values of layer 1, transposed
    float *b1p = nullptr;                  // [m1p]
    float *b2p = nullptr;                  // [m2p]
    // batched-GEMM path of any depth: layer l padded to Np[l] outputs (multiple
    // of 128) x Kp[l] inputs (multiple of 64), zeros in the padding
    int Kp[NQS_MAX_LAYERS] = {0}, Np[NQS_MAX_LAYERS] = {0};
    void *Wd[NQS_MAX_LAYERS] = {nullptr};  // [Np][Kp] bf16/f16/e4m3 codes, or FP32 values
    float *bd[NQS_MAX_LAYERS] = {nullptr}; // [Np]
    // E4M3 copy: layer l computes z = (sum_k qW qA) acc_scale[l] + b, acc_scale = weight scale x input
    // scale (the input scale a power of two, 1 for the spins), and stores the next layer's input as the
    // code of ReLU(z) next_inv[l] (next_inv = 1 / the next input scale).  1 in the other formats.
    float acc_scale[NQS_MAX_LAYERS] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
    float next_inv[NQS_MAX_LAYERS] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
};

// Residual convolutional network copy in one sampling format: one FP32 array
// of the rounded parameters in the order of the parameter vector, each
// convolution's weights rearranged as [in channel][3x3 offset][out channel].
struct CnnDev {
    int L = 0, F = 0, R = 0, dtype = 1;
    float *p = nullptr;
    int64_t w0 = 0, b0 = 0, gf = 0, bef = 0;
    int64_t g[NQS_MAX_LAYERS] = {0}, be[NQS_MAX_LAYERS] = {0}, w1[NQS_MAX_LAYERS] = {0}, b1[NQS_MAX_LAYERS] = {0},
            w2[NQS_MAX_LAYERS] = {0}, b2[NQS_MAX_LAYERS] = {0};
    // matrix-core operands: block r's conv1 (j = 0) and conv2 (j = 1) weights at
    // wmc + (2 r + j) 9 F^2 elements, laid out [offset][out channel][in channel];
    // raw BF16/FP16 codes for those copies, FP32 values for the FP32 copy
    void *wmc = nullptr;
};

// Complex-parameter RBM copy: FP32 (real, imaginary) pairs of the rounded
// parameters and the tables (cosh 2W, sinh 2W) as (re, im, re, im).
struct CrbmDev {
    int N = 0, M = 0;
    float2 *a = nullptr;      // [N]
    float *a2 = nullptr;      // [N]  4 Re(a_i) / ln 2
    float2 *b = nullptr;      // [M]
    float2 *Wt = nullptr;     // [N][M]  Wt[i][j] = W[j][i]
    float4 *CS = nullptr;     // [N][M] + one neutral entry (1, 0, 0, 0) at N*M
    float4 *CSt = nullptr;    // [M][N]
};

struct Copy {
    bool valid = false;
    RbmDev rbm;
    FfnnDev ffnn;
    CnnDev cnn;
    CrbmDev crbm;
    void *block = nullptr;   // single allocation backing the arrays above
};

}  // namespace nqs

struct nqs_model {
    nqs_model_desc desc{};
    int64_t P = 0;
    int device = 0;
    double *master = nullptr;           // FP64 master parameters on the device
    nqs::Copy copies[5];                // indexed by nqs_dtype
    float *wb_f32 = nullptr;            // scratch FP32 rounded parameter vector [P]
    // the dense-network sampler's captured sweep: executable graph, the event after its last
    // replay, and the launch arguments it was captured with
    hipGraphExec_t sweep_exec = nullptr;
    hipEvent_t sweep_done = nullptr;
    std::string sweep_sig;
};

namespace nqs {

// Kernels that take more than 64 KiB of dynamic LDS must say so before launch.
template <typename Kern>
static inline void allow_lds(Kern k, size_t bytes)
{
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

// FP8 (E4M3) copy of one tensor with its per-tensor scale amax/448; `amax` is
// one 64-bit word of device scratch.
nqs_status launch_e4m3_tensor(const double *src, int64_t n, unsigned long long *amax, float *dst, hipStream_t stream);

// Zero n 64-bit words with a kernel (usable inside captured graphs).
nqs_status launch_zero_u64(void *p, int64_t n, hipStream_t stream);

// Compute units of the current device (cached per device).
int device_cus();
// A stream of the current device that only records captures (never runs work).
hipStream_t capture_stream();

// Per-device growable scratch (never shrinks; freed at process exit).
void *workspace(size_t bytes, hipStream_t stream);
// Slot 1 is for entry points that hold vectors across calls into others
// (which use slot 0).
constexpr int kWorkspaceSlots = 3;
void *workspace_slot(int slot, size_t bytes, hipStream_t stream);
// low-precision Cholesky factor of T + shift and its inverse (srmix.hip)
size_t mix_workspace_bytes(int64_t n);
nqs_status mix_factor(const float *T, int64_t n, double shift, int fmt, void *ws, float **Lin, float **LinT,
                      int64_t *np_out, unsigned long long *nfix, hipStream_t s);

int64_t model_num_params(const nqs_model_desc &d);

// Build (or rebuild) the `dtype` copy of the model on `stream`.
nqs_status ensure_copy(nqs_model *m, int dtype, hipStream_t stream);

// kernels -------------------------------------------------------------------
nqs_status launch_downcast(const double *src, int64_t n, int dtype, float *dst, float *scale_out,
                           hipStream_t stream);
nqs_status rbm_build_copy(nqs_model *m, int dtype, hipStream_t stream);
// noise_sigma > 0: the noisy target; dg_*: the run-time detectors (all three per-chain arrays, or none)
nqs_status rbm_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples,
                      float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream,
                      double noise_sigma = 0.0, uint64_t noise_seed = 0, unsigned long long *dg_nonfinite = nullptr,
                      uint32_t *dg_stuck = nullptr, float *dg_drift = nullptr);

// Sampler launch (one translation unit per lanes-per-chain G).
struct RbmSampleArgs {
    RbmDev net;
    int8_t *chain_state;
    int8_t *samples;
    float *logpsi;
    unsigned long long *n_acc;
    int64_t n_chains;
    int n_sweeps, n_burnin, sweep_size, refresh_sweeps;
    uint64_t seed, step_offset;
    uint32_t inst, chain_id_offset;
    int n_traced;
    int32_t *tr_site;
    uint32_t *tr_ubits;
    float *tr_delta;
    uint8_t *tr_acc;
    // noisy target: log pi~(x) = log pi(x) + sigma g(x), g(x) standard normal fixed per x
    float noise_sigma;
    uint32_t noise_key0, noise_key1;
    // run-time detectors (the traced instantiation; all NULL or all set), per chain: proposals with a
    // non-finite log-ratio, the longest run of sweeps without an accepted move, the largest
    // |log psi carried by the accepted log-ratios - log psi recomputed from theta| at a refresh
    unsigned long long *dg_nonfinite;
    uint32_t *dg_stuck;
    float *dg_drift;
};
struct RbmLaunch {
    int K, threads, blocks;
    bool lds, trace, noise;
    int init;              // 1: draw the start states inside the kernel (flip moves)
    size_t lds_bytes;
};
nqs_status rbm_sample_checked(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples,
                              float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, nqs_sample_diag *diag,
                              hipStream_t stream);

// Launch plan of the RBM sampler: lanes per chain G, units per lane K, chains
// per block, table placement.
struct RbmPlan {
    int G, K, cpb;
    bool lds;
    size_t tab_bytes;
    bool tuned;
    float tuned_ms;
};
// lds_req: -1 = LDS when the table fits, 0 = through L2, 1 = LDS; cpb_req 0 = spread over every CU
nqs_status rbm_plan_rule(int N, int M, int64_t n_chains, int G, int lds_req, int cpb_req, RbmPlan *P);
nqs_status rbm_plan_tuned(nqs_model *m, const nqs_sample_cfg &cfg, const int *Gs, int nG, hipStream_t stream,
                          RbmPlan *out);
nqs_status rbm_launch_plan(const RbmSampleArgs &A, const RbmPlan &P, bool trace, bool noise, int init,
                           hipStream_t stream);
nqs_status rbm_sample_launch_g16(const RbmSampleArgs &A, const RbmLaunch &L, hipStream_t s);
nqs_status rbm_sample_launch_g32(const RbmSampleArgs &A, const RbmLaunch &L, hipStream_t s);
nqs_status rbm_sample_launch_g64(const RbmSampleArgs &A, const RbmLaunch &L, hipStream_t s);
nqs_status rbm_sample_batched(const nqs_sample_job *jobs, int n_jobs, int mode, hipStream_t stream);
nqs_status rbm_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                            double *eloc, hipStream_t stream);
// O holds parameter columns [p0, p1) (row stride p1 - p0); the full matrix is p0 = 0, p1 = P
nqs_status rbm_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                           const float *vjp_in, float *vjp_out, hipStream_t stream, int64_t p0, int64_t p1);
nqs_status ffnn_build_copy(nqs_model *m, int dtype, hipStream_t stream);
// complex-parameter RBM
nqs_status crbm_build_copy(nqs_model *m, int dtype, hipStream_t stream);
// complex RBM: log-derivatives O[n][2P'] (real parts, then imaginary parts) and Re log psi; the real
// 2n x 2n embedding of T = Obar Obar^H / n; the centred right-hand side (Re eps, Im eps) of the complex
// solve (library workspace); the SR update from y[2n] = (Re z, Im z)
nqs_status crbm_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                            hipStream_t stream);
nqs_status cplx_gram_embedded(const float *O, int64_t n, int64_t P, float *T2, hipStream_t stream);
nqs_status cplx_sr_rhs(const double *eloc_re, const double *eloc_im, int64_t n, double **e2, hipStream_t stream);
nqs_status crbm_sr_update(nqs_model *m, const int8_t *samples, int64_t n, const double *y, double lr, double *master,
                          hipStream_t stream);
nqs_status crbm_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                       uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream);
nqs_status crbm_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                             double *eloc_re, double *eloc_im, hipStream_t stream);
// residual convolutional network
int64_t cnn_num_params(int F, int R);
nqs_status cnn_build_copy(nqs_model *m, int dtype, hipStream_t stream);
nqs_status cnn_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                      uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream);
nqs_status cnn_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                            double *eloc, hipStream_t stream);
nqs_status cnn_logpsi(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, hipStream_t stream);
nqs_status cnn_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                           const float *vjp_in, float *vjp_out, hipStream_t stream);
// vjp_out[p] (+)= sum_k g[k] O[k][p] over a block of rows of O (first: overwrite)
nqs_status launch_vjp_chunk(const float *O, const float *g, int64_t n, int64_t P, float *out, bool first,
                            hipStream_t stream);
nqs_status ffnn_sample(nqs_model *m, const nqs_sample_cfg &cfg, int8_t *chain_state, int8_t *samples,
                       float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, hipStream_t stream);
nqs_status ffnn_local_energy(nqs_model *m, const nqs_ham_desc &ham, const int8_t *samples, int64_t n, int dtype,
                             double *eloc, hipStream_t stream);
nqs_status ffnn_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                            const float *vjp_in, float *vjp_out, hipStream_t stream, int64_t p0, int64_t p1);
// T of the samples, column blocks of `chunk` parameters expanded from per-sample
// activations and deltas computed once
nqs_status ffnn_sample_gram(nqs_model *m, const int8_t *samples, int64_t n, int64_t chunk, float *T,
                            hipStream_t stream);
nqs_status launch_init_chains(int8_t *chain_state, int64_t n_chains, int N, int move, uint64_t seed,
                              uint32_t inst, int64_t chain_id_offset, hipStream_t stream);
nqs_status launch_energy_stats(const double *eloc, int64_t n, int64_t n_chains, double *stats, hipStream_t stream);
// the same with the file-scope scratch (kStatsScratchDoubles doubles per device; no allocation)
constexpr int64_t kStatsScratchDoubles = 131072;
nqs_status launch_energy_stats_noalloc(const double *eloc, int64_t n, int64_t n_chains, double *stats,
                                       hipStream_t stream);
nqs_status launch_forces(const float *O, const double *eloc, int64_t n, int64_t P, double *F, double *Omean,
                         hipStream_t stream);
// One layer of factors of O for the factored sample-space Gram matrix:
// O_layer(k) = U_k (x) V_k and U_k, plus V_k when c = 1 (all FP32, row-major).
struct FacLayerDesc {
    const float *U, *V;
    int64_t ldu, ldv;
    int du, dv, c;
};
size_t fac_workspace_bytes(const FacLayerDesc *lay, int L, int64_t n);
nqs_status launch_fac_gram(const FacLayerDesc *lay, int L, int64_t n, float *T, void *ws, hipStream_t stream);
void launch_spins_to_f32(const int8_t *s, int64_t count, float *out, hipStream_t stream);
// factors of an RBM: t = tanh(theta) [n][M]
nqs_status rbm_tanh_theta(nqs_model *m, const int8_t *samples, int64_t n, float *t, hipStream_t stream);
// factors of a dense network: layer inputs a_{l-1} [n][sum of inputs] and deltas [n][sum of outputs]
nqs_status ffnn_factors(nqs_model *m, const int8_t *samples, int64_t n, float *acts, float *dels, hipStream_t stream);

// mode 0 S, 1 T, 2 T accumulated into `out`; the _ws form takes a caller-carved
// workspace of gram_workspace_bytes(n, P) bytes
nqs_status launch_gram(const float *O, int64_t n, int64_t P, int mode, float *out, hipStream_t stream);
size_t gram_workspace_bytes(int64_t n, int64_t P);
nqs_status launch_gram_ws(const float *O, int64_t n, int64_t P, int mode, float *out, void *ws, hipStream_t stream);

}  // namespace nqs
