// Many RBM instances of uneven size in one persistent launch.
//
// Work items are (instance, 4 chains) pairs, sorted by decreasing cost
// (chains x proposals x hidden units per lane) and handed out through a global
// counter, so the largest instances start first and small ones fill the
// gaps (longest-processing-time-first list scheduling).  Every chain group
// uses 64 lanes; the hidden units per lane K of each instance is resolved at
// run time by a uniform branch into the same per-chain code the single-
// instance sampler runs, so results are identical to a separate launch with
// 64 lanes per chain.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "rbm_sampler.h"

namespace nqs {

struct BatchJob {
    RbmSampleArgs A;
    int K;
    int lds;       // 1: the (C,S) table fits in LDS
    int init;
    int pad;
};

constexpr int kBatchThreads = 256;   // 4 chains of 64 lanes per work item
constexpr int kBatchKMax = 16;

template <bool LDS>
__device__ __forceinline__ void batched_dispatch(const RbmSampleArgs &A, int K, int64_t c, int gl, const float2 *s_tab,
                                                 bool init)
{
    switch (K) {
#define NQS_BK(KK) \
    case KK: rbm_run_chain<64, KK, LDS, false>(A, c, gl, s_tab, init); break;
        NQS_BK(1) NQS_BK(2) NQS_BK(3) NQS_BK(4) NQS_BK(5) NQS_BK(6) NQS_BK(7) NQS_BK(8)
        NQS_BK(9) NQS_BK(10) NQS_BK(11) NQS_BK(12) NQS_BK(13) NQS_BK(14) NQS_BK(15) NQS_BK(16)
#undef NQS_BK
    default: break;
    }
}

__global__ void __launch_bounds__(kBatchThreads) rbm_batched_kernel(const BatchJob *__restrict__ jobs,
                                                                     const int2 *__restrict__ items, int n_items,
                                                                     int *counter)
{
    extern __shared__ float2 s_tab[];
    __shared__ int s_item;
    int loaded = -1;
    const int gl = threadIdx.x & 63;
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
        const int64_t c = (int64_t)w.y + (threadIdx.x >> 6);
        if (c < J.A.n_chains) {
            if (J.lds) batched_dispatch<true>(J.A, J.K, c, gl, s_tab, J.init != 0);
            else batched_dispatch<false>(J.A, J.K, c, gl, s_tab, J.init != 0);
        }
        __syncthreads();   // the LDS table may be replaced by the next item
    }
}

__global__ void zero_int_kernel(int *p)
{
    *p = 0;
}

nqs_status rbm_sample_batched(const nqs_sample_job *jobs, int n_jobs, int mode, hipStream_t stream)
{
    // validate and prepare every instance before any launch
    for (int k = 0; k < n_jobs; ++k) {
        const nqs_sample_job &j = jobs[k];
        if (!j.model || !j.chain_state) return set_error(NQS_EINVAL, "job without model or chain_state");
        if (j.model->desc.arch != NQS_RBM) return set_error(NQS_EUNSUPPORTED, "batched sampling is implemented for RBMs");
        if (j.cfg.move != NQS_MOVE_FLIP) return set_error(NQS_EUNSUPPORTED, "batched sampling uses single-flip moves");
        if (j.cfg.dtype != NQS_F32 && j.cfg.dtype != NQS_F16 && j.cfg.dtype != NQS_BF16)
            return set_error(NQS_EINVAL, "batched sampling dtype must be F32, F16 or BF16");
        if (j.cfg.n_chains < 0 || j.cfg.n_sweeps < 0 || j.cfg.n_burnin < 0) return set_error(NQS_EINVAL, "negative sizes");
        if (j.cfg.chain_id_offset < 0 || j.cfg.chain_id_offset + j.cfg.n_chains > ((int64_t)1 << 32))
            return set_error(NQS_EINVAL, "global chain ids must fit in 32 bits");
        nqs_status st = ensure_copy(j.model, j.cfg.dtype, stream);
        if (st != NQS_OK) return st;
        const RbmDev &net = j.model->copies[j.cfg.dtype].rbm;
        if (!(net.max_abs_w <= 5.0f)) return set_error(NQS_EUNSUPPORTED, "the product-form RBM sampler needs |W| <= 5");
        if ((net.M + 63) / 64 > kBatchKMax) return set_error(NQS_EUNSUPPORTED, "hidden width > 1024 in a batched job");
        if ((net.N + 31) / 32 > 64) return set_error(NQS_EUNSUPPORTED, "too many sites in a batched job");
    }
    if (mode == 1) {
        // one specialised launch per instance, in order, on the same stream
        for (int k = 0; k < n_jobs; ++k) {
            nqs_sample_cfg cfg = jobs[k].cfg;
            cfg.lanes_per_chain = 64;
            nqs_status st = rbm_sample(jobs[k].model, cfg, jobs[k].chain_state, jobs[k].samples, jobs[k].logpsi,
                                       jobs[k].n_accepted, nullptr, stream);
            if (st != NQS_OK) return st;
        }
        return NQS_OK;
    }
    std::vector<BatchJob> bj(n_jobs);
    std::vector<int2> items;
    std::vector<double> cost;
    size_t lds_need = 0;
    for (int k = 0; k < n_jobs; ++k) {
        const nqs_sample_job &j = jobs[k];
        const RbmDev &net = j.model->copies[j.cfg.dtype].rbm;
        RbmSampleArgs &A = bj[k].A;
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
        A.n_traced = 0;
        A.noise_sigma = 0.0f;
        A.noise_key0 = A.noise_key1 = 0u;
        A.tr_site = nullptr;
        A.tr_ubits = nullptr;
        A.tr_delta = nullptr;
        A.tr_acc = nullptr;
        bj[k].K = (net.M + 63) / 64;
        const size_t tab = sizeof(float2) * ((size_t)net.N * net.M + 1);
        bj[k].lds = tab <= 160 * 1024 ? 1 : 0;
        bj[k].init = j.cfg.init_chains ? 1 : 0;
        if (bj[k].lds) lds_need = std::max(lds_need, tab);
        const double props = (double)(j.cfg.n_burnin + j.cfg.n_sweeps) * A.sweep_size;
        for (int64_t c = 0; c < j.cfg.n_chains; c += kBatchThreads / 64) {
            items.push_back(make_int2(k, (int)c));
            cost.push_back(props * (bj[k].K + 2) * (bj[k].lds ? 1.0 : 1.5));
        }
    }
    if (items.empty()) return NQS_OK;
    std::vector<int> order(items.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<int2> sorted(items.size());
    for (size_t q = 0; q < order.size(); ++q) sorted[q] = items[order[q]];

    const size_t bytes_jobs = sizeof(BatchJob) * n_jobs, bytes_items = sizeof(int2) * sorted.size();
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

}  // namespace nqs
