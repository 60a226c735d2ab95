// Instantiations of the dense-network sampler and local-energy kernels.
#include "ffnn_mc.h"

namespace nqs {

template <typename T, int QK>
static void launch_sample_tq(bool trace, const FfnnSampleArgs &A, int blocks, size_t lds, hipStream_t s)
{
    if (trace) {
        allow_lds(ffnn_sample_kernel<T, QK, true>, lds);
        hipLaunchKernelGGL((ffnn_sample_kernel<T, QK, true>), dim3(blocks), dim3(256), lds, s, A);
    } else {
        allow_lds(ffnn_sample_kernel<T, QK, false>, lds);
        hipLaunchKernelGGL((ffnn_sample_kernel<T, QK, false>), dim3(blocks), dim3(256), lds, s, A);
    }
}

template <typename T>
static bool launch_sample_t(int QK, bool trace, const FfnnSampleArgs &A, int blocks, size_t lds, hipStream_t s)
{
    switch (QK) {
    case 1: launch_sample_tq<T, 1>(trace, A, blocks, lds, s); return true;
    case 2: launch_sample_tq<T, 2>(trace, A, blocks, lds, s); return true;
    case 3: launch_sample_tq<T, 3>(trace, A, blocks, lds, s); return true;
    case 4: launch_sample_tq<T, 4>(trace, A, blocks, lds, s); return true;
    case 5: launch_sample_tq<T, 5>(trace, A, blocks, lds, s); return true;
    case 6: launch_sample_tq<T, 6>(trace, A, blocks, lds, s); return true;
    case 7: launch_sample_tq<T, 7>(trace, A, blocks, lds, s); return true;
    case 8: launch_sample_tq<T, 8>(trace, A, blocks, lds, s); return true;
    default: return false;
    }
}

nqs_status ffnn_sample_dispatch(int dtype, int QK, bool trace, const FfnnSampleArgs &A, int blocks, size_t lds,
                                hipStream_t s)
{
    bool ok;
    if (dtype == NQS_F32) ok = launch_sample_t<float>(QK, trace, A, blocks, lds, s);
    else if (dtype == NQS_F16) ok = launch_sample_t<_Float16>(QK, trace, A, blocks, lds, s);
    else ok = launch_sample_t<__bf16>(QK, trace, A, blocks, lds, s);
    if (!ok) return set_error(NQS_EUNSUPPORTED, "first hidden width not supported by the sampler");
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

template <typename T, int QK>
static void launch_eloc_tq(const FfnnElocArgs &A, int blocks, size_t lds, hipStream_t s)
{
    allow_lds(ffnn_eloc_kernel<T, QK>, lds);
    hipLaunchKernelGGL((ffnn_eloc_kernel<T, QK>), dim3(blocks), dim3(256), lds, s, A);
}

template <typename T>
static bool launch_eloc_t(int QK, const FfnnElocArgs &A, int blocks, size_t lds, hipStream_t s)
{
    switch (QK) {
    case 1: launch_eloc_tq<T, 1>(A, blocks, lds, s); return true;
    case 2: launch_eloc_tq<T, 2>(A, blocks, lds, s); return true;
    case 3: launch_eloc_tq<T, 3>(A, blocks, lds, s); return true;
    case 4: launch_eloc_tq<T, 4>(A, blocks, lds, s); return true;
    case 5: launch_eloc_tq<T, 5>(A, blocks, lds, s); return true;
    case 6: launch_eloc_tq<T, 6>(A, blocks, lds, s); return true;
    case 7: launch_eloc_tq<T, 7>(A, blocks, lds, s); return true;
    case 8: launch_eloc_tq<T, 8>(A, blocks, lds, s); return true;
    default: return false;
    }
}

nqs_status ffnn_eloc_dispatch(int dtype, int QK, const FfnnElocArgs &A, int blocks, size_t lds, hipStream_t s)
{
    bool ok;
    if (dtype == NQS_F32) ok = launch_eloc_t<float>(QK, A, blocks, lds, s);
    else if (dtype == NQS_F16) ok = launch_eloc_t<_Float16>(QK, A, blocks, lds, s);
    else ok = launch_eloc_t<__bf16>(QK, A, blocks, lds, s);
    if (!ok) return set_error(NQS_EUNSUPPORTED, "first hidden width not supported by the local-energy kernel");
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
