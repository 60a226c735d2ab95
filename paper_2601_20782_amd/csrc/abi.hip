// C entry points of libnqs: argument validation, model handles, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "nqs.h"

namespace nqs {

static thread_local std::string g_last_error;

nqs_status set_error(nqs_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

nqs_status hip_error(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(e == hipErrorOutOfMemory ? NQS_ENOMEM : NQS_EDEVICE, m);
}

// ---------------------------------------------------------------------------
// Per-device workspace
// ---------------------------------------------------------------------------
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
static std::mutex g_ws_mutex;
static std::vector<Workspace> g_ws;   // [device * kWorkspaceSlots + slot]

hipStream_t capture_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) streams[dev] = nullptr;
    return streams[dev];
}

int device_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    static std::mutex mu;
    static std::vector<int> cache;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

void *workspace_slot(int slot, size_t bytes, hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || slot < 0 || slot >= kWorkspaceSlots) return nullptr;
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    const size_t idx = (size_t)dev * kWorkspaceSlots + slot;
    if (g_ws.size() <= idx) g_ws.resize(idx + 1);
    Workspace &w = g_ws[idx];
    if (w.bytes < bytes) {
        if (w.ptr) {
            // the old buffer may still be in use by earlier work on `stream`
            if (hipStreamSynchronize(stream) != hipSuccess) return nullptr;
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
        if (hipMalloc(&w.ptr, want) != hipSuccess) return nullptr;
        w.bytes = want;
    }
    return w.ptr;
}

void *workspace(size_t bytes, hipStream_t stream) { return workspace_slot(0, bytes, stream); }

int64_t model_num_params(const nqs_model_desc &d)
{
    const int64_t N = d.n_visible;
    if (d.arch == NQS_RBM) return N + d.widths[0] + (int64_t)d.widths[0] * N;
    if (d.arch == NQS_RESCNN) return cnn_num_params(d.widths[0], d.n_layers);
    if (d.arch == NQS_CRBM) return 2 * (N + d.widths[0] + (int64_t)d.widths[0] * N);
    int64_t p = 0, prev = N;
    for (int l = 0; l < d.n_layers; ++l) {
        p += (int64_t)d.widths[l] * (prev + 1);
        prev = d.widths[l];
    }
    return p;
}

nqs_status ensure_copy(nqs_model *m, int dtype, hipStream_t stream)
{
    if (m->copies[dtype].valid) return NQS_OK;
    if (m->desc.arch == NQS_RBM) return rbm_build_copy(m, dtype, stream);
    if (m->desc.arch == NQS_RESCNN) return cnn_build_copy(m, dtype, stream);
    if (m->desc.arch == NQS_CRBM) return crbm_build_copy(m, dtype, stream);
    return ffnn_build_copy(m, dtype, stream);
}

static void invalidate(nqs_model *m)
{
    for (auto &c : m->copies) c.valid = false;
}

static nqs_status validate_desc(const nqs_model_desc *d)
{
    if (!d) return set_error(NQS_EINVAL, "desc is NULL");
    if (d->n_visible < 2 || d->n_visible > 4096) return set_error(NQS_EINVAL, "n_visible must be in [2, 4096]");
    if (d->arch == NQS_RBM || d->arch == NQS_CRBM) {
        if (d->n_layers != 1) return set_error(NQS_EINVAL, "RBM needs n_layers = 1");
        if (d->arch == NQS_CRBM && d->marshall) return set_error(NQS_EINVAL, "the complex RBM carries its own phases");
        if (d->widths[0] < 1 || d->widths[0] > 8192) return set_error(NQS_EINVAL, "RBM hidden width must be in [1, 8192]");
    } else if (d->arch == NQS_FFNN) {
        if (d->n_layers < 1 || d->n_layers > NQS_MAX_LAYERS) return set_error(NQS_EINVAL, "FFNN needs 1..8 layers");
        for (int l = 0; l < d->n_layers; ++l)
            if (d->widths[l] < 1 || d->widths[l] > 8192) return set_error(NQS_EINVAL, "FFNN widths must be in [1, 8192]");
    } else if (d->arch == NQS_RESCNN) {
        if (d->lat_dim != 2 || d->lat_L < 3 || (int64_t)d->lat_L * d->lat_L != d->n_visible)
            return set_error(NQS_EINVAL, "convolutional network needs lat_dim = 2, lat_L >= 3, n_visible = lat_L^2");
        if (d->widths[0] < 1 || d->widths[0] > 256) return set_error(NQS_EINVAL, "filters (widths[0]) must be in [1, 256]");
        if (d->n_layers < 0 || d->n_layers > NQS_MAX_LAYERS) return set_error(NQS_EINVAL, "residual blocks must be 0..8");
        if (d->marshall) return set_error(NQS_EUNSUPPORTED, "no Marshall sign for the convolutional network");
    } else {
        return set_error(NQS_EINVAL, "unknown arch");
    }
    if (d->marshall) {
        if (d->lat_dim != 1 && d->lat_dim != 2) return set_error(NQS_EINVAL, "Marshall sign needs lat_dim 1 or 2");
        const int64_t n = d->lat_dim == 1 ? d->lat_L : (int64_t)d->lat_L * d->lat_L;
        if (n != d->n_visible) return set_error(NQS_EINVAL, "Marshall lattice size does not match n_visible");
    }
    return NQS_OK;
}

static bool all_finite(const double *p, int64_t n)
{
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(p[k])) return false;
    return true;
}

static int ham_sites(const nqs_ham_desc &h)
{
    return h.dim == 1 ? h.L : h.L * h.L;
}

}  // namespace nqs

using namespace nqs;

extern "C" {

const char *nqs_last_error(void)
{
    return g_last_error.c_str();
}

const char *nqs_version(void)
{
    return "libnqs 0.1 (gfx950)";
}

int64_t nqs_model_num_params(const nqs_model *m)
{
    return m ? m->P : -1;
}

nqs_status nqs_model_create(const nqs_model_desc *desc, const double *host_params, int64_t n_params, nqs_model **out)
{
    if (!out) return set_error(NQS_EINVAL, "out is NULL");
    *out = nullptr;
    nqs_status st = validate_desc(desc);
    if (st != NQS_OK) return st;
    const int64_t P = model_num_params(*desc);
    if (n_params != P) return set_error(NQS_EINVAL, "n_params does not match the architecture (expected " + std::to_string(P) + ")");
    if (!host_params) return set_error(NQS_EINVAL, "host_params is NULL");
    if (!all_finite(host_params, P)) return set_error(NQS_ENUMERIC, "parameters contain NaN or Inf");
    nqs_model *m = new nqs_model();
    m->desc = *desc;
    m->P = P;
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; return set_error(NQS_EDEVICE, "no HIP device"); }
    hipError_t e = hipMalloc(&m->master, sizeof(double) * P);
    if (e != hipSuccess) { delete m; return hip_error(e, "hipMalloc(master)"); }
    e = hipMalloc(&m->wb_f32, sizeof(float) * P);
    if (e != hipSuccess) { (void)hipFree(m->master); delete m; return hip_error(e, "hipMalloc(scratch)"); }
    e = hipMemcpy(m->master, host_params, sizeof(double) * P, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(m->master); (void)hipFree(m->wb_f32); delete m; return hip_error(e, "hipMemcpy(master)"); }
    *out = m;
    return NQS_OK;
}

nqs_status nqs_model_set_params(nqs_model *m, const double *host_params, int64_t n_params)
{
    if (!m || !host_params) return set_error(NQS_EINVAL, "NULL argument");
    if (n_params != m->P) return set_error(NQS_EINVAL, "n_params does not match the model");
    if (!all_finite(host_params, n_params)) return set_error(NQS_ENUMERIC, "parameters contain NaN or Inf");
    NQS_HIP_TRY(hipDeviceSynchronize());
    NQS_HIP_TRY(hipMemcpy(m->master, host_params, sizeof(double) * n_params, hipMemcpyHostToDevice));
    invalidate(m);
    return NQS_OK;
}

nqs_status nqs_model_set_params_device(nqs_model *m, const double *dev_params, int64_t n_params, void *stream)
{
    if (!m || !dev_params) return set_error(NQS_EINVAL, "NULL argument");
    if (n_params != m->P) return set_error(NQS_EINVAL, "n_params does not match the model");
    hipStream_t s = (hipStream_t)stream;
    NQS_HIP_TRY(hipMemcpyAsync(m->master, dev_params, sizeof(double) * n_params, hipMemcpyDeviceToDevice, s));
    invalidate(m);
    return NQS_OK;
}

nqs_status nqs_model_destroy(nqs_model *m)
{
    if (!m) return NQS_OK;
    (void)hipDeviceSynchronize();
    if (m->sweep_exec) (void)hipGraphExecDestroy(m->sweep_exec);
    if (m->sweep_done) (void)hipEventDestroy(m->sweep_done);
    for (auto &c : m->copies)
        if (c.block) (void)hipFree(c.block);
    (void)hipFree(m->master);
    (void)hipFree(m->wb_f32);
    delete m;
    return NQS_OK;
}

nqs_status nqs_model_prepare(nqs_model *m, int32_t dtype, void *stream)
{
    if (!m) return set_error(NQS_EINVAL, "NULL model");
    if (dtype < NQS_F32 || dtype > NQS_FP8_E4M3) return set_error(NQS_EINVAL, "dtype must be F32, F16, BF16 or FP8_E4M3");
    m->copies[dtype].valid = false;
    return ensure_copy(m, dtype, (hipStream_t)stream);
}

nqs_status nqs_downcast(const double *src, int64_t n, int32_t dtype, float *dst, float *scale_out, void *stream)
{
    if (n < 0) return set_error(NQS_EINVAL, "n < 0");
    if (n == 0) return NQS_OK;
    if (!src || !dst) return set_error(NQS_EINVAL, "NULL src/dst");
    if (dtype < NQS_F64 || dtype > NQS_FP8_E4M3) return set_error(NQS_EINVAL, "unknown dtype");
    return launch_downcast(src, n, dtype, dst, scale_out, (hipStream_t)stream);
}

// Argument checks shared by nqs_sample and nqs_sample_checked (n_chains > 0 here).
static nqs_status check_sample_args(const nqs_model *m, const nqs_sample_cfg &c, const int8_t *chain_state,
                                    const nqs_trace *trace)
{
    const int N = m->desc.n_visible;
    if (!chain_state) return set_error(NQS_EINVAL, "chain_state is NULL");
    if (c.n_chains > (int64_t)1 << 31) return set_error(NQS_EINVAL, "n_chains too large");
    if (c.move != NQS_MOVE_FLIP && c.move != NQS_MOVE_EXCHANGE) return set_error(NQS_EINVAL, "unknown move");
    if (c.move == NQS_MOVE_EXCHANGE && (N % 2 != 0)) return set_error(NQS_EINVAL, "exchange moves need an even number of sites");
    if (c.sweep_size < 0) return set_error(NQS_EINVAL, "sweep_size < 0");
    if (c.instance_id >= (1u << 24)) return set_error(NQS_EINVAL, "instance_id must fit in 24 bits");
    if (c.lanes_per_chain != 0 && c.lanes_per_chain != 16 && c.lanes_per_chain != 32 && c.lanes_per_chain != 64 &&
        !(c.lanes_per_chain == -1 && (m->desc.arch == NQS_FFNN || m->desc.arch == NQS_RESCNN)) &&
        !(c.lanes_per_chain == NQS_LANES_TUNED && m->desc.arch == NQS_RBM))
        return set_error(NQS_EINVAL, "lanes_per_chain must be 0, 16, 32 or 64 (-1 for a dense network, "
                                     "NQS_LANES_TUNED for an RBM)");
    if (c.dtype != NQS_F32 && c.dtype != NQS_F16 && c.dtype != NQS_BF16 && c.dtype != NQS_FP8_E4M3)
        return set_error(NQS_EINVAL, "sampling dtype must be F32, F16, BF16 or FP8_E4M3");
    if (c.chain_id_offset < 0 || c.chain_id_offset + c.n_chains > ((int64_t)1 << 32))
        return set_error(NQS_EINVAL, "global chain ids must fit in 32 bits");
    if (trace && trace->n_chains_traced > 0) {
        if (!trace->site || !trace->ubits || !trace->delta || !trace->accepted)
            return set_error(NQS_EINVAL, "trace buffers are NULL");
        if (trace->n_chains_traced > c.n_chains) return set_error(NQS_EINVAL, "n_chains_traced > n_chains");
    }
    return NQS_OK;
}

nqs_status nqs_sample(nqs_model *m, const nqs_sample_cfg *cfg, int8_t *chain_state, int8_t *samples, float *logpsi,
                      uint64_t *n_accepted, const nqs_trace *trace, void *stream)
{
    if (!m || !cfg) return set_error(NQS_EINVAL, "NULL model or cfg");
    const nqs_sample_cfg &c = *cfg;
    if (c.n_chains < 0 || c.n_sweeps < 0 || c.n_burnin < 0) return set_error(NQS_EINVAL, "negative sizes");
    if (c.n_chains == 0) return NQS_OK;
    nqs_status st = check_sample_args(m, c, chain_state, trace);
    if (st != NQS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (m->desc.arch == NQS_RBM) {
        if (c.move != NQS_MOVE_FLIP) return set_error(NQS_EUNSUPPORTED, "the RBM sampler implements single-flip moves");
        return rbm_sample(m, c, chain_state, samples, logpsi, n_accepted, trace, s);
    }
    if (m->desc.arch == NQS_CRBM) {
        if (c.move != NQS_MOVE_FLIP) return set_error(NQS_EUNSUPPORTED, "the complex RBM sampler implements single flips");
        return crbm_sample(m, c, chain_state, samples, logpsi, n_accepted, trace, s);
    }
    if (m->desc.arch == NQS_RESCNN) {
        if (c.move != NQS_MOVE_FLIP || c.sweep_size != 0)
            return set_error(NQS_EUNSUPPORTED, "the convolutional-network sampler implements single flips, sweeps of N");
        if (c.dtype == NQS_FP8_E4M3) return set_error(NQS_EUNSUPPORTED, "no FP8 copy of the convolutional network");
        return cnn_sample(m, c, chain_state, samples, logpsi, n_accepted, trace, s);
    }
    return ffnn_sample(m, c, chain_state, samples, logpsi, n_accepted, trace, s);
}

nqs_status nqs_sample_checked(nqs_model *m, const nqs_sample_cfg *cfg, int8_t *chain_state, int8_t *samples,
                              float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, nqs_sample_diag *diag,
                              void *stream)
{
    if (!m || !cfg || !diag) return set_error(NQS_EINVAL, "NULL model, cfg or diag");
    const nqs_sample_cfg &c = *cfg;
    if (c.n_chains < 0 || c.n_sweeps < 0 || c.n_burnin < 0) return set_error(NQS_EINVAL, "negative sizes");
    if (diag->stuck_after < 0) return set_error(NQS_EINVAL, "stuck_after < 0");
    diag->total_nonfinite = 0;
    diag->chains_stuck = 0;
    diag->max_drift = 0.0f;
    if (c.n_chains == 0) return NQS_OK;
    nqs_status st = check_sample_args(m, c, chain_state, trace);
    if (st != NQS_OK) return st;
    if (m->desc.arch != NQS_RBM || c.move != NQS_MOVE_FLIP)
        return set_error(NQS_EUNSUPPORTED, "the run-time detectors are built into the RBM single-flip sampler");
    return rbm_sample_checked(m, c, chain_state, samples, logpsi, n_accepted, trace, diag, (hipStream_t)stream);
}

nqs_status nqs_sample_noisy(nqs_model *m, const nqs_sample_cfg *cfg, double noise_sigma, uint64_t noise_seed,
                            int8_t *chain_state, int8_t *samples, float *logpsi, uint64_t *n_accepted, void *stream)
{
    if (!m || !cfg) return set_error(NQS_EINVAL, "NULL model or cfg");
    if (!(noise_sigma >= 0.0) || !std::isfinite(noise_sigma)) return set_error(NQS_EINVAL, "noise_sigma must be finite and >= 0");
    if (m->desc.arch != NQS_RBM || cfg->move != NQS_MOVE_FLIP)
        return set_error(NQS_EUNSUPPORTED, "the noisy target is implemented for the RBM with single flips");
    if (m->desc.n_visible > 128) return set_error(NQS_EUNSUPPORTED, "the noisy target takes at most 128 sites");
    if (noise_sigma == 0.0) return nqs_sample(m, cfg, chain_state, samples, logpsi, n_accepted, nullptr, stream);
    // the same argument checks as nqs_sample, then the noisy kernels
    const nqs_sample_cfg &c = *cfg;
    if (c.n_chains < 0 || c.n_sweeps < 0 || c.n_burnin < 0) return set_error(NQS_EINVAL, "negative sizes");
    if (c.n_chains == 0) return NQS_OK;
    if (!chain_state) return set_error(NQS_EINVAL, "chain_state is NULL");
    if (c.n_chains > (int64_t)1 << 31) return set_error(NQS_EINVAL, "n_chains too large");
    if (c.sweep_size < 0) return set_error(NQS_EINVAL, "sweep_size < 0");
    if (c.instance_id >= (1u << 24)) return set_error(NQS_EINVAL, "instance_id must fit in 24 bits");
    if (c.lanes_per_chain != 0 && c.lanes_per_chain != 16 && c.lanes_per_chain != 32 && c.lanes_per_chain != 64)
        return set_error(NQS_EINVAL, "lanes_per_chain must be 0, 16, 32 or 64");
    if (c.dtype != NQS_F32 && c.dtype != NQS_F16 && c.dtype != NQS_BF16 && c.dtype != NQS_FP8_E4M3)
        return set_error(NQS_EINVAL, "sampling dtype must be F32, F16, BF16 or FP8_E4M3");
    if (c.chain_id_offset < 0 || c.chain_id_offset + c.n_chains > ((int64_t)1 << 32))
        return set_error(NQS_EINVAL, "global chain ids must fit in 32 bits");
    return rbm_sample(m, c, chain_state, samples, logpsi, n_accepted, nullptr, (hipStream_t)stream, noise_sigma,
                      noise_seed);
}

nqs_status nqs_sample_plan(nqs_model *m, const nqs_sample_cfg *cfg, nqs_launch_plan *plan, void *stream)
{
    if (!m || !cfg || !plan) return set_error(NQS_EINVAL, "NULL model, cfg or plan");
    if (m->desc.arch != NQS_RBM) return set_error(NQS_EUNSUPPORTED, "launch plans describe the RBM sampler");
    const nqs_sample_cfg &c = *cfg;
    if (c.n_chains <= 0 || c.n_chains > (int64_t)1 << 31) return set_error(NQS_EINVAL, "n_chains must be in [1, 2^31]");
    if (c.dtype != NQS_F32 && c.dtype != NQS_F16 && c.dtype != NQS_BF16 && c.dtype != NQS_FP8_E4M3)
        return set_error(NQS_EINVAL, "sampling dtype must be F32, F16, BF16 or FP8_E4M3");
    if (c.lanes_per_chain != 0 && c.lanes_per_chain != 16 && c.lanes_per_chain != 32 && c.lanes_per_chain != 64 &&
        c.lanes_per_chain != NQS_LANES_TUNED)
        return set_error(NQS_EINVAL, "lanes_per_chain must be 0, 16, 32, 64 or NQS_LANES_TUNED");
    hipStream_t s = (hipStream_t)stream;
    nqs_status st = ensure_copy(m, c.dtype, s);
    if (st != NQS_OK) return st;
    RbmPlan P;
    st = c.lanes_per_chain == NQS_LANES_TUNED
             ? rbm_plan_tuned(m, c, nullptr, 0, s, &P)
             : rbm_plan_rule(m->desc.n_visible, m->desc.widths[0], c.n_chains, c.lanes_per_chain, -1, 0, &P);
    if (st != NQS_OK) return st;
    plan->lanes_per_chain = P.G;
    plan->units_per_lane = P.K;
    plan->chains_per_block = P.cpb;
    plan->table_in_lds = P.lds ? 1 : 0;
    plan->tuned = P.tuned ? 1 : 0;
    plan->tuned_ms = P.tuned_ms;
    return NQS_OK;
}

nqs_status nqs_sample_batched(const nqs_sample_job *jobs, int32_t n_jobs, int32_t mode, void *stream)
{
    if (n_jobs < 0) return set_error(NQS_EINVAL, "n_jobs < 0");
    if (n_jobs == 0) return NQS_OK;
    if (!jobs) return set_error(NQS_EINVAL, "jobs is NULL");
    if (mode != 0 && mode != 1) return set_error(NQS_EINVAL, "mode must be 0 (persistent) or 1 (one launch per job)");
    return rbm_sample_batched(jobs, n_jobs, mode, (hipStream_t)stream);
}

nqs_status nqs_local_energy(nqs_model *m, const nqs_ham_desc *ham, const int8_t *samples, int64_t n_samples,
                            int32_t eval_dtype, double *eloc, void *stream)
{
    if (!m || !ham) return set_error(NQS_EINVAL, "NULL model or hamiltonian");
    if (n_samples < 0) return set_error(NQS_EINVAL, "n_samples < 0");
    if (n_samples == 0) return NQS_OK;
    if (!samples || !eloc) return set_error(NQS_EINVAL, "NULL samples/eloc");
    const nqs_ham_desc &h = *ham;
    if (h.kind != NQS_TFIM && h.kind != NQS_HEISENBERG) return set_error(NQS_EINVAL, "unknown hamiltonian");
    if (h.dim != 1 && h.dim != 2) return set_error(NQS_EINVAL, "dim must be 1 or 2");
    if (h.pbc && h.L < 3) return set_error(NQS_EINVAL, "periodic lattices need L >= 3");
    if (!h.pbc && h.L < 2) return set_error(NQS_EINVAL, "L >= 2 required");
    if (ham_sites(h) != m->desc.n_visible) return set_error(NQS_EINVAL, "lattice size does not match n_visible");
    if (eval_dtype != NQS_F32 && eval_dtype != NQS_F16 && eval_dtype != NQS_BF16 && eval_dtype != NQS_FP8_E4M3)
        return set_error(NQS_EINVAL, "eval dtype must be F32, F16, BF16 or FP8_E4M3");
    hipStream_t s = (hipStream_t)stream;
    if (m->desc.arch == NQS_RBM) {
        return rbm_local_energy(m, h, samples, n_samples, eval_dtype, eloc, s);
    }
    if (m->desc.arch == NQS_RESCNN) return cnn_local_energy(m, h, samples, n_samples, eval_dtype, eloc, s);
    if (m->desc.arch == NQS_CRBM) return crbm_local_energy(m, h, samples, n_samples, eval_dtype, eloc, nullptr, s);
    return ffnn_local_energy(m, h, samples, n_samples, eval_dtype, eloc, s);
}

nqs_status nqs_local_energy_complex(nqs_model *m, const nqs_ham_desc *ham, const int8_t *samples, int64_t n_samples,
                                   int32_t eval_dtype, double *eloc_re, double *eloc_im, void *stream)
{
    if (!m || !ham) return set_error(NQS_EINVAL, "NULL model or hamiltonian");
    if (m->desc.arch != NQS_CRBM) {
        // real amplitudes: the real part validates the arguments; the imaginary part is zero
        const nqs_status st = nqs_local_energy(m, ham, samples, n_samples, eval_dtype, eloc_re, stream);
        if (st != NQS_OK || !eloc_im || n_samples <= 0) return st;
        return launch_zero_u64(reinterpret_cast<uint64_t *>(eloc_im), n_samples, (hipStream_t)stream);
    }
    if (n_samples < 0) return set_error(NQS_EINVAL, "n_samples < 0");
    if (n_samples == 0) return NQS_OK;
    if (!samples || !eloc_re || !eloc_im) return set_error(NQS_EINVAL, "NULL samples/eloc_re/eloc_im");
    const nqs_ham_desc &h = *ham;
    if (h.dim != 1 && h.dim != 2) return set_error(NQS_EINVAL, "dim must be 1 or 2");
    if (h.pbc && h.L < 3) return set_error(NQS_EINVAL, "periodic lattices need L >= 3");
    if (!h.pbc && h.L < 2) return set_error(NQS_EINVAL, "L >= 2 required");
    if (ham_sites(h) != m->desc.n_visible) return set_error(NQS_EINVAL, "lattice size does not match n_visible");
    if (eval_dtype != NQS_F32 && eval_dtype != NQS_F16 && eval_dtype != NQS_BF16)
        return set_error(NQS_EINVAL, "eval dtype must be F32, F16 or BF16");
    return crbm_local_energy(m, h, samples, n_samples, eval_dtype, eloc_re, eloc_im, (hipStream_t)stream);
}

nqs_status nqs_energy_stats(const double *eloc, int64_t n, int64_t n_chains, double *stats, void *stream)
{
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!eloc || !stats) return set_error(NQS_EINVAL, "NULL eloc/stats");
    if (n_chains < 0) return set_error(NQS_EINVAL, "n_chains < 0");
    return launch_energy_stats(eloc, n, n_chains, stats, (hipStream_t)stream);
}

nqs_status nqs_energy_stats_noalloc(const double *eloc, int64_t n, int64_t n_chains, double *stats, void *stream)
{
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!eloc || !stats) return set_error(NQS_EINVAL, "NULL eloc/stats");
    if (n_chains < 0) return set_error(NQS_EINVAL, "n_chains < 0");
    return launch_energy_stats_noalloc(eloc, n, n_chains, stats, (hipStream_t)stream);
}

nqs_status nqs_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                           const float *vjp_in, float *vjp_out, void *stream)
{
    if (!m) return set_error(NQS_EINVAL, "NULL model");
    if (n < 0) return set_error(NQS_EINVAL, "n < 0");
    if (n == 0) return NQS_OK;
    if (!samples) return set_error(NQS_EINVAL, "NULL samples");
    if ((vjp_in == nullptr) != (vjp_out == nullptr)) return set_error(NQS_EINVAL, "vjp_in and vjp_out go together");
    hipStream_t s = (hipStream_t)stream;
    if (m->desc.arch == NQS_CRBM) {
        if (vjp_in) return set_error(NQS_EUNSUPPORTED, "the vector-Jacobian product of the complex RBM is not built");
        return crbm_logpsi_grad(m, samples, n, logpsi, O, s);
    }
    if (m->desc.arch == NQS_RESCNN) {
        if (!O && !vjp_in) return logpsi ? cnn_logpsi(m, samples, n, logpsi, s) : NQS_OK;
        return cnn_logpsi_grad(m, samples, n, logpsi, O, vjp_in, vjp_out, s);
    }
    if (m->desc.arch == NQS_RBM) return rbm_logpsi_grad(m, samples, n, logpsi, O, vjp_in, vjp_out, s, 0, m->P);
    return ffnn_logpsi_grad(m, samples, n, logpsi, O, vjp_in, vjp_out, s, 0, m->P);
}

nqs_status nqs_logpsi_grad_cols(nqs_model *m, const int8_t *samples, int64_t n, int64_t p0, int64_t p1, float *O,
                                void *stream)
{
    if (m && m->desc.arch == NQS_CRBM)
        return set_error(NQS_EUNSUPPORTED, "column blocks of the complex RBM's log-derivatives are not built");
    if (m && m->desc.arch == NQS_RESCNN)
        return set_error(NQS_EUNSUPPORTED, "log-derivatives of the convolutional network are not built");
    if (!m) return set_error(NQS_EINVAL, "NULL model");
    if (n < 0) return set_error(NQS_EINVAL, "n < 0");
    if (p0 < 0 || p1 <= p0 || p1 > m->P) return set_error(NQS_EINVAL, "need 0 <= p0 < p1 <= P");
    if (n == 0) return NQS_OK;
    if (!samples || !O) return set_error(NQS_EINVAL, "NULL samples/O");
    hipStream_t s = (hipStream_t)stream;
    if (m->desc.arch == NQS_RBM) return rbm_logpsi_grad(m, samples, n, nullptr, O, nullptr, nullptr, s, p0, p1);
    return ffnn_logpsi_grad(m, samples, n, nullptr, O, nullptr, nullptr, s, p0, p1);
}

nqs_status nqs_sample_gram_factored(nqs_model *m, const int8_t *samples, int64_t n, float *T, void *stream)
{
    if (m && m->desc.arch == NQS_CRBM)
        return set_error(NQS_EUNSUPPORTED, "column blocks of the complex RBM's log-derivatives are not built");
    if (m && m->desc.arch == NQS_RESCNN)
        return set_error(NQS_EUNSUPPORTED, "log-derivatives of the convolutional network are not built");
    if (!m) return set_error(NQS_EINVAL, "NULL model");
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!samples || !T) return set_error(NQS_EINVAL, "NULL samples/T");
    hipStream_t s = (hipStream_t)stream;
    const nqs_model_desc &d = m->desc;
    FacLayerDesc lay[NQS_MAX_LAYERS];
    int L = 0;
    size_t fbytes = 0;
    int64_t sa = 0, sd = 0;
    if (d.arch == NQS_RBM) {
        L = 1;
        fbytes = sizeof(float) * (size_t)n * (size_t)(d.n_visible + d.widths[0]);
    } else {
        L = d.n_layers;
        for (int l = 0; l < L; ++l) {
            sa += l == 0 ? d.n_visible : d.widths[l - 1];
            sd += d.widths[l];
        }
        fbytes = sizeof(float) * (size_t)n * (size_t)(sa + sd);
    }
    fbytes = (fbytes + 255) & ~(size_t)255;
    // the factor layout is fixed before the workspace size is known: fill the
    // descriptors with offsets first, then rebase them on the workspace
    if (d.arch == NQS_RBM) {
        const int N = d.n_visible, M = d.widths[0];
        lay[0] = FacLayerDesc{nullptr, nullptr, M, N, M, N, 1};
    } else {
        int64_t oa = 0, od = 0;
        for (int l = 0; l < L; ++l) {
            const int in = l == 0 ? d.n_visible : d.widths[l - 1], out = d.widths[l];
            lay[l] = FacLayerDesc{(const float *)(uintptr_t)(od * sizeof(float)),
                                  (const float *)(uintptr_t)(oa * sizeof(float)), sd, sa, out, in, 0};
            oa += in;
            od += out;
        }
    }
    char *ws = (char *)workspace(fbytes + fac_workspace_bytes(lay, L, n), s);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    nqs_status st = NQS_OK;
    if (d.arch == NQS_RBM) {
        const int N = d.n_visible;
        float *t = (float *)ws, *sf = t + (size_t)n * d.widths[0];
        st = rbm_tanh_theta(m, samples, n, t, s);
        if (st != NQS_OK) return st;
        launch_spins_to_f32(samples, n * N, sf, s);
        lay[0].U = t;
        lay[0].V = sf;
    } else {
        float *dels = (float *)ws, *acts = dels + (size_t)n * sd;
        st = ffnn_factors(m, samples, n, acts, dels, s);
        if (st != NQS_OK) return st;
        for (int l = 0; l < L; ++l) {
            lay[l].U = dels + (uintptr_t)lay[l].U / sizeof(float);
            lay[l].V = acts + (uintptr_t)lay[l].V / sizeof(float);
        }
    }
    return launch_fac_gram(lay, L, n, T, ws + fbytes, s);
}

nqs_status nqs_sample_gram(nqs_model *m, const int8_t *samples, int64_t n, int64_t chunk_params, float *T,
                           void *stream)
{
    if (m && m->desc.arch == NQS_CRBM)
        return set_error(NQS_EUNSUPPORTED, "column blocks of the complex RBM's log-derivatives are not built");
    if (m && m->desc.arch == NQS_RESCNN) {
        // weights shared across sites: O is formed whole (one block of all columns)
        if (n <= 0 || !samples || !T) return set_error(NQS_EINVAL, "bad samples/T");
        hipStream_t s = (hipStream_t)stream;
        const size_t ob = (sizeof(float) * (size_t)n * (size_t)m->P + 255) & ~(size_t)255;
        if (ob > ((size_t)1 << 32)) return set_error(NQS_EUNSUPPORTED, "O of the convolutional network over 4 GiB");
        char *ws = (char *)workspace_slot(1, ob, s);
        if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
        nqs_status st = cnn_logpsi_grad(m, samples, n, nullptr, (float *)ws, nullptr, nullptr, s);
        if (st != NQS_OK) return st;
        return launch_gram((const float *)ws, n, m->P, 1, T, s);
    }
    if (!m) return set_error(NQS_EINVAL, "NULL model");
    if (n <= 0) return set_error(NQS_EINVAL, "n must be positive");
    if (!samples || !T) return set_error(NQS_EINVAL, "NULL samples/T");
    if (chunk_params < 0) return set_error(NQS_EINVAL, "chunk_params < 0");
    const int64_t P = m->P;
    int64_t chunk = chunk_params;
    if (chunk == 0) {
        // automatic: a column block of at most 1 GiB, a multiple of the contraction step
        chunk = std::max<int64_t>(32, ((int64_t)(1ll << 28) / n) & ~(int64_t)31);
    }
    chunk = std::min(chunk, P);
    hipStream_t s = (hipStream_t)stream;
    if (m->desc.arch != NQS_RBM) return ffnn_sample_gram(m, samples, n, chunk, T, s);
    // RBM: each block of O is recomputed from the samples (theta is cheap next to the block)
    const size_t oc_bytes = (sizeof(float) * (size_t)n * (size_t)chunk + 255) & ~(size_t)255;
    char *ws = (char *)workspace(oc_bytes + gram_workspace_bytes(n, chunk), (hipStream_t)stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    float *Oc = (float *)ws;
    for (int64_t p0 = 0; p0 < P; p0 += chunk) {
        const int64_t p1 = std::min(P, p0 + chunk);
        nqs_status st = rbm_logpsi_grad(m, samples, n, nullptr, Oc, nullptr, nullptr, s, p0, p1);
        if (st != NQS_OK) return st;
        st = launch_gram_ws(Oc, n, p1 - p0, p0 == 0 ? 1 : 2, T, ws + oc_bytes, s);
        if (st != NQS_OK) return st;
    }
    return NQS_OK;
}

nqs_status nqs_forces(const float *O, const double *eloc, int64_t n, int64_t P, double *F, double *Omean, void *stream)
{
    if (n <= 0 || P <= 0) return set_error(NQS_EINVAL, "n and P must be positive");
    if (!O || !eloc || !F) return set_error(NQS_EINVAL, "NULL O/eloc/F");
    return launch_forces(O, eloc, n, P, F, Omean, (hipStream_t)stream);
}

nqs_status nqs_gram(const float *O, int64_t n, int64_t P, int32_t mode, float *out, void *stream)
{
    if (n <= 0 || P <= 0) return set_error(NQS_EINVAL, "n and P must be positive");
    if (!O || !out) return set_error(NQS_EINVAL, "NULL O/out");
    if (mode < 0 || mode > 3) return set_error(NQS_EINVAL, "mode must be 0 (S), 1 (T), 2 (T accumulate) or 3 (complex T)");
    if (mode == 3) {
        if (P % 2 != 0) return set_error(NQS_EINVAL, "mode 3 takes O as [n][2P'] (real parts, then imaginary parts)");
        return cplx_gram_embedded(O, n, P, out, (hipStream_t)stream);
    }
    return launch_gram(O, n, P, mode, out, (hipStream_t)stream);
}

}  // extern "C"
