// Many RBM instances of uneven size in one persistent launch.
//
// Work items are (instance, 256 / G chains) pairs, sorted by decreasing cost
// (proposals x hidden units per lane, more for a table read through L2) and
// handed out through a global counter, so the largest instances start first
// and small ones fill the gaps (longest-processing-time-first list
// scheduling).  Each instance keeps its own lanes per chain G (32 for M <= 256,
// else 64, or the tuner's choice between them) and units per lane K; a
// uniform branch on (G, K, table placement) enters the same per-chain code the
// single-instance sampler runs, so every instance's results equal those of a
// separate launch with the same G.  Traced chains record their decisions as in
// a single launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rbm_sampler.h"

namespace nqs {

struct BatchJob {
    RbmSampleArgs A;
    int G, K;
    int lds;       // 1: the (C,S) table fits in LDS
    int init;
};

constexpr int kBatchThreads = 256;   // one work item: 256 / G chains
constexpr int kBatchK32 = 8;         // G = 32 serves M <= 256
constexpr int kBatchK64 = 16;        // G = 64 serves M <= 1024

template <int G, bool LDS>
__device__ __forceinline__ void batched_dispatch(const RbmSampleArgs &A, int K, int64_t c, int gl, const float2 *s_tab,
                                                 bool init)
{
    switch (K) {
#define NQS_BK(KK) \
    case KK: rbm_run_chain<G, KK, LDS, true>(A, c, gl, s_tab, init); break;
        NQS_BK(1) NQS_BK(2) NQS_BK(3) NQS_BK(4) NQS_BK(5) NQS_BK(6) NQS_BK(7) NQS_BK(8)
#undef NQS_BK
    default:
        if constexpr (G == 64) {
            switch (K) {
#define NQS_BK(KK) \
    case KK: rbm_run_chain<64, KK, LDS, true>(A, c, gl, s_tab, init); break;
                NQS_BK(9) NQS_BK(10) NQS_BK(11) NQS_BK(12) NQS_BK(13) NQS_BK(14) NQS_BK(15) NQS_BK(16)
#undef NQS_BK
            default: break;
            }
        }
        break;
    }
}

__global__ void __launch_bounds__(kBatchThreads) rbm_batched_kernel(const BatchJob *__restrict__ jobs,
                                                                     const int2 *__restrict__ items, int n_items,
                                                                     int *counter)
{
    extern __shared__ float2 s_tab[];
    __shared__ int s_item;
    int loaded = -1;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;   // every block reaches this once the list is exhausted
        const int2 w = items[it];
        const BatchJob &J = jobs[w.x];
        if (J.lds && w.x != loaded) {
            const int total = J.A.net.N * J.A.net.M + 1;
            for (int k = threadIdx.x; k < total; k += kBatchThreads) s_tab[k] = J.A.net.CS[k];
            __syncthreads();
            loaded = w.x;
        }
        const int G = J.G;   // uniform over the block
        const int gl = threadIdx.x & (G - 1);
        const int64_t c = (int64_t)w.y + threadIdx.x / G;
        if (c < J.A.n_chains) {
            const bool init = J.init != 0;
            if (G == 32) {
                if (J.lds) batched_dispatch<32, true>(J.A, J.K, c, gl, s_tab, init);
                else batched_dispatch<32, false>(J.A, J.K, c, gl, s_tab, init);
            } else {
                if (J.lds) batched_dispatch<64, true>(J.A, J.K, c, gl, s_tab, init);
                else batched_dispatch<64, false>(J.A, J.K, c, gl, s_tab, init);
            }
        }
        __syncthreads();   // the LDS table may be replaced by the next item
    }
}

__global__ void zero_int_kernel(int *p)
{
    *p = 0;
}

// Lanes per chain of one batched instance: the request (32 or 64), else 32
// when K = ceil(M / 32) <= 8 and 64 above.  A tuned request returns 0 here:
// the whole batch decides those (batch_tune).
static bool lanes_ok(int N, int M, int G)
{
    return G == 32 ? (M + 31) / 32 <= kBatchK32 && (N + 31) / 32 <= 32 : (M + 63) / 64 <= kBatchK64 && (N + 31) / 32 <= 64;
}

static nqs_status batched_lanes(const nqs_model *m, const nqs_sample_cfg &cfg, int *G)
{
    const int N = m->desc.n_visible, M = m->desc.widths[0];
    if (cfg.lanes_per_chain == 32 || cfg.lanes_per_chain == 64) {
        *G = cfg.lanes_per_chain;
        if (!lanes_ok(N, M, *G))
            return set_error(NQS_EUNSUPPORTED, "batched sampling: 32 lanes serve M <= 256, 64 lanes M <= 1024");
        return NQS_OK;
    }
    if (cfg.lanes_per_chain != 0 && cfg.lanes_per_chain != NQS_LANES_TUNED)
        return set_error(NQS_EINVAL, "batched sampling takes lanes_per_chain 0, 32, 64 or NQS_LANES_TUNED");
    if (!lanes_ok(N, M, 32) && !lanes_ok(N, M, 64))
        return set_error(NQS_EUNSUPPORTED, "hidden width > 1024 or too many sites in a batched job");
    *G = cfg.lanes_per_chain == NQS_LANES_TUNED && lanes_ok(N, M, 32) && lanes_ok(N, M, 64) ? 0
                                                                                           : (lanes_ok(N, M, 32) ? 32 : 64);
    return NQS_OK;
}

static BatchJob make_batch_job(const nqs_sample_job &j, int G)
{
    BatchJob b;
    const RbmDev &net = j.model->copies[j.cfg.dtype].rbm;
    RbmSampleArgs &A = b.A;
    std::memset(&A, 0, sizeof(A));
    A.net = net;
    A.chain_state = j.chain_state;
    A.samples = j.samples;
    A.logpsi = j.logpsi;
    A.n_acc = (unsigned long long *)j.n_accepted;
    A.n_chains = j.cfg.n_chains;
    A.n_sweeps = j.cfg.n_sweeps;
    A.n_burnin = j.cfg.n_burnin;
    A.sweep_size = j.cfg.sweep_size > 0 ? j.cfg.sweep_size : net.N;
    A.refresh_sweeps = j.cfg.refresh_sweeps > 0 ? j.cfg.refresh_sweeps : 1;
    A.seed = j.cfg.seed;
    A.step_offset = j.cfg.step_offset;
    A.inst = j.cfg.instance_id;
    A.chain_id_offset = (uint32_t)j.cfg.chain_id_offset;
    const bool tr = j.trace && j.trace->n_chains_traced > 0;
    A.n_traced = tr ? j.trace->n_chains_traced : 0;
    A.tr_site = tr ? j.trace->site : nullptr;
    A.tr_ubits = tr ? j.trace->ubits : nullptr;
    A.tr_delta = tr ? j.trace->delta : nullptr;
    A.tr_acc = tr ? j.trace->accepted : nullptr;
    b.G = G;
    b.K = (net.M + G - 1) / G;
    b.lds = sizeof(float2) * ((size_t)net.N * net.M + 1) <= 160 * 1024 ? 1 : 0;
    b.init = j.cfg.init_chains ? 1 : 0;
    return b;
}

// The persistent launch of a prepared batch: work items sorted by decreasing
// cost, descriptors staged in the workspace (the stream is synchronised once).
static nqs_status launch_batch(const std::vector<BatchJob> &bj, hipStream_t stream)
{
    std::vector<int2> items;
    std::vector<double> cost;
    size_t lds_need = 0;
    for (size_t k = 0; k < bj.size(); ++k) {
        const BatchJob &b = bj[k];
        if (b.lds) lds_need = std::max(lds_need, sizeof(float2) * ((size_t)b.A.net.N * b.A.net.M + 1));
        const double props = (double)(b.A.n_burnin + b.A.n_sweeps) * b.A.sweep_size;
        const int per_item = kBatchThreads / b.G;
        for (int64_t c = 0; c < b.A.n_chains; c += per_item) {
            items.push_back(make_int2((int)k, (int)c));
            cost.push_back(props * (b.K + 2) * (b.lds ? 1.0 : 1.5));
        }
    }
    if (items.empty()) return NQS_OK;
    std::vector<int> order(items.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<int2> sorted(items.size());
    for (size_t q = 0; q < order.size(); ++q) sorted[q] = items[order[q]];

    const size_t bytes_jobs = sizeof(BatchJob) * bj.size(), bytes_items = sizeof(int2) * sorted.size();
    char *ws = (char *)workspace(bytes_jobs + bytes_items + 256, stream);
    if (!ws) return set_error(NQS_ENOMEM, "workspace allocation failed");
    BatchJob *d_jobs = (BatchJob *)ws;
    int2 *d_items = (int2 *)(ws + ((bytes_jobs + 15) & ~(size_t)15));
    int *d_counter = (int *)(ws + ((bytes_jobs + 15) & ~(size_t)15) + ((bytes_items + 15) & ~(size_t)15));
    NQS_HIP_TRY(hipMemcpyAsync(d_jobs, bj.data(), bytes_jobs, hipMemcpyHostToDevice, stream));
    NQS_HIP_TRY(hipMemcpyAsync(d_items, sorted.data(), bytes_items, hipMemcpyHostToDevice, stream));
    NQS_HIP_TRY(hipStreamSynchronize(stream));   // the host vectors go out of scope
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, stream, d_counter);
    const int cus = device_cus();
    const int per_cu = lds_need > 80 * 1024 ? 1 : (lds_need > 40 * 1024 ? 2 : 4);
    const int grid = (int)std::min<size_t>(sorted.size(), (size_t)cus * per_cu);
    allow_lds(rbm_batched_kernel, lds_need);
    hipLaunchKernelGGL(rbm_batched_kernel, dim3(grid), dim3(kBatchThreads), lds_need, stream, d_jobs, d_items,
                       (int)sorted.size(), d_counter);
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

// Lanes per chain of the tuned instances, decided for the whole batch: the
// persistent launch is timed on a short burn-in from fresh states in scratch
// memory (no outputs) with the tuned instances at 32 lanes where allowed,
// all at 64, and at each instance's single-launch choice between the two
// (rbm_plan_tuned); the fastest assignment is kept for the life of the
// process, keyed by the batch's (device, N, M, dtype, n_chains, request) list.
namespace {
std::mutex g_batch_mu;
std::map<std::vector<int64_t>, std::vector<int>> g_batch_tune;
}

static nqs_status batch_tune(const nqs_sample_job *jobs, int n_jobs, std::vector<int> &lanes, hipStream_t stream)
{
    std::vector<int> tuned;
    for (int k = 0; k < n_jobs; ++k)
        if (lanes[k] == 0) tuned.push_back(k);
    if (tuned.empty()) return NQS_OK;
    int dev = 0;
    NQS_HIP_TRY(hipGetDevice(&dev));
    std::vector<int64_t> key{dev};
    for (int k = 0; k < n_jobs; ++k) {
        const nqs_sample_job &j = jobs[k];
        key.insert(key.end(), {j.model->desc.n_visible, j.model->desc.widths[0], j.cfg.dtype, j.cfg.n_chains, lanes[k]});
    }
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        auto it = g_batch_tune.find(key);
        if (it != g_batch_tune.end()) {
            lanes = it->second;
            return NQS_OK;
        }
    }
    // candidate assignments of the tuned instances
    std::vector<std::vector<int>> cand(3, lanes);
    for (int k : tuned) {
        cand[0][k] = 32;
        cand[1][k] = 64;
        static const int both[2] = {32, 64};
        RbmPlan P;
        nqs_status st = rbm_plan_tuned(jobs[k].model, jobs[k].cfg, both, 2, stream, &P);
        if (st != NQS_OK) return st;
        cand[2][k] = P.G;
    }
    // scratch states and a burn-in of ~2e7 proposals over the batch
    int64_t per_sweep = 0, bytes = 0;
    std::vector<int64_t> off(n_jobs);
    for (int k = 0; k < n_jobs; ++k) {
        const int N = jobs[k].model->desc.n_visible;
        off[k] = bytes;
        bytes += (jobs[k].cfg.n_chains * N + 255) & ~(int64_t)255;
        per_sweep += jobs[k].cfg.n_chains * N;
    }
    const int sweeps = (int)std::max<int64_t>(1, std::min<int64_t>(64, (20000000 + per_sweep - 1) / std::max<int64_t>(1, per_sweep)));
    int8_t *scratch = nullptr;
    NQS_HIP_TRY(hipMalloc(&scratch, (size_t)std::max<int64_t>(bytes, 256)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nqs_status result = NQS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventCreate failed");
    int best = 0;
    float best_ms = 3.4e38f;
    for (int q = 0; q < 3 && result == NQS_OK; ++q) {
        if (q == 2 && (cand[2] == cand[0] || cand[2] == cand[1])) continue;
        std::vector<BatchJob> bj(n_jobs);
        for (int k = 0; k < n_jobs; ++k) {
            nqs_sample_job j = jobs[k];
            j.chain_state = scratch + off[k];
            j.samples = nullptr;
            j.logpsi = nullptr;
            j.n_accepted = nullptr;
            j.trace = nullptr;
            j.cfg.n_sweeps = 0;
            j.cfg.n_burnin = sweeps;
            j.cfg.init_chains = 1;
            bj[k] = make_batch_job(j, cand[q][k]);
        }
        float t = 3.4e38f;
        for (int rep = 0; rep < 3 && result == NQS_OK; ++rep) {   // the first run warms up
            if (hipEventRecord(e0, stream) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventRecord failed");
            if (result == NQS_OK) result = launch_batch(bj, stream);
            if (result == NQS_OK && hipEventRecord(e1, stream) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventRecord failed");
            if (result == NQS_OK && hipEventSynchronize(e1) != hipSuccess) result = set_error(NQS_EDEVICE, "tuning run failed");
            float ms = 0.0f;
            if (result == NQS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) result = set_error(NQS_EDEVICE, "hipEventElapsedTime failed");
            if (rep > 0) t = std::min(t, ms);
        }
        if (result == NQS_OK && t < best_ms) {
            best_ms = t;
            best = q;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (result != NQS_OK) return result;
    lanes = cand[best];
    std::lock_guard<std::mutex> lock(g_batch_mu);
    g_batch_tune[key] = lanes;
    return NQS_OK;
}

nqs_status rbm_sample_batched(const nqs_sample_job *jobs, int n_jobs, int mode, hipStream_t stream)
{
    // validate and prepare every instance before any launch
    std::vector<int> lanes(n_jobs);
    for (int k = 0; k < n_jobs; ++k) {
        const nqs_sample_job &j = jobs[k];
        if (!j.model || !j.chain_state) return set_error(NQS_EINVAL, "job without model or chain_state");
        if (j.model->desc.arch != NQS_RBM) return set_error(NQS_EUNSUPPORTED, "batched sampling is implemented for RBMs");
        if (j.cfg.move != NQS_MOVE_FLIP) return set_error(NQS_EUNSUPPORTED, "batched sampling uses single-flip moves");
        if (j.cfg.dtype != NQS_F32 && j.cfg.dtype != NQS_F16 && j.cfg.dtype != NQS_BF16)
            return set_error(NQS_EINVAL, "batched sampling dtype must be F32, F16 or BF16");
        if (j.cfg.n_chains < 0 || j.cfg.n_sweeps < 0 || j.cfg.n_burnin < 0) return set_error(NQS_EINVAL, "negative sizes");
        if (j.cfg.sweep_size < 0) return set_error(NQS_EINVAL, "sweep_size < 0");
        if (j.cfg.n_chains > (int64_t)1 << 31) return set_error(NQS_EINVAL, "n_chains too large");
        if (j.cfg.instance_id >= (1u << 24)) return set_error(NQS_EINVAL, "instance_id must fit in 24 bits");
        if (j.cfg.chain_id_offset < 0 || j.cfg.chain_id_offset + j.cfg.n_chains > ((int64_t)1 << 32))
            return set_error(NQS_EINVAL, "global chain ids must fit in 32 bits");
        if (j.trace && j.trace->n_chains_traced > 0) {
            if (!j.trace->site || !j.trace->ubits || !j.trace->delta || !j.trace->accepted)
                return set_error(NQS_EINVAL, "trace buffers are NULL");
            if (j.trace->n_chains_traced > j.cfg.n_chains) return set_error(NQS_EINVAL, "n_chains_traced > n_chains");
        }
        nqs_status st = ensure_copy(j.model, j.cfg.dtype, stream);
        if (st != NQS_OK) return st;
        const RbmDev &net = j.model->copies[j.cfg.dtype].rbm;
        if (!(net.max_abs_w <= 5.0f)) return set_error(NQS_EUNSUPPORTED, "the product-form RBM sampler needs |W| <= 5");
        st = batched_lanes(j.model, j.cfg, &lanes[k]);
        if (st != NQS_OK) return st;
    }
    nqs_status st = batch_tune(jobs, n_jobs, lanes, stream);
    if (st != NQS_OK) return st;
    if (mode == 1) {
        // one specialised launch per instance, in order, on the same stream, at the instance's lanes per chain
        for (int k = 0; k < n_jobs; ++k) {
            nqs_sample_cfg cfg = jobs[k].cfg;
            cfg.lanes_per_chain = lanes[k];
            st = rbm_sample(jobs[k].model, cfg, jobs[k].chain_state, jobs[k].samples, jobs[k].logpsi,
                            jobs[k].n_accepted, jobs[k].trace, stream);
            if (st != NQS_OK) return st;
        }
        return NQS_OK;
    }
    std::vector<BatchJob> bj(n_jobs);
    for (int k = 0; k < n_jobs; ++k) bj[k] = make_batch_job(jobs[k], lanes[k]);
    return launch_batch(bj, stream);
}

}  // namespace nqs
