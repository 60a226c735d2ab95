// Instantiations of the register-resident dense-network kernels (16-bit operands).
#include "ffnn_reg.h"

namespace nqs {

template <typename T, int KF>
static void launch_reg_sample(bool trace, const FfnnSampleArgs &A, int blocks, size_t lds, hipStream_t s)
{
    if (trace) {
        allow_lds(ffnn_sample_reg_kernel<T, KF, true>, lds);
        hipLaunchKernelGGL((ffnn_sample_reg_kernel<T, KF, true>), dim3(blocks), dim3(kRegThreads), lds, s, A);
    } else {
        allow_lds(ffnn_sample_reg_kernel<T, KF, false>, lds);
        hipLaunchKernelGGL((ffnn_sample_reg_kernel<T, KF, false>), dim3(blocks), dim3(kRegThreads), lds, s, A);
    }
}

template <typename T>
static bool reg_sample_t(int KF, bool trace, const FfnnSampleArgs &A, int blocks, size_t lds, hipStream_t s)
{
    switch (KF) {
    case 8: launch_reg_sample<T, 8>(trace, A, blocks, lds, s); return true;
    case 12: launch_reg_sample<T, 12>(trace, A, blocks, lds, s); return true;
    case 16: launch_reg_sample<T, 16>(trace, A, blocks, lds, s); return true;
    case 20: launch_reg_sample<T, 20>(trace, A, blocks, lds, s); return true;
    case 24: launch_reg_sample<T, 24>(trace, A, blocks, lds, s); return true;
    case 28: launch_reg_sample<T, 28>(trace, A, blocks, lds, s); return true;
    case 32: launch_reg_sample<T, 32>(trace, A, blocks, lds, s); return true;
    default: return false;
    }
}

size_t ffnn_reg_sample_lds(int dtype, int N, int m1p, int m2p)
{
    return dtype == NQS_F16 ? RegSampleLds<_Float16>::bytes(N, m1p, m2p) : RegSampleLds<__bf16>::bytes(N, m1p, m2p);
}

nqs_status ffnn_reg_sample_dispatch(int dtype, bool trace, const FfnnSampleArgs &A, int blocks, size_t lds,
                                    hipStream_t s)
{
    const int KF = A.net.m1p / 16;
    const bool ok = dtype == NQS_F16 ? reg_sample_t<_Float16>(KF, trace, A, blocks, lds, s)
                                     : reg_sample_t<__bf16>(KF, trace, A, blocks, lds, s);
    if (!ok) return set_error(NQS_EUNSUPPORTED, "first hidden width not supported by the register-resident sampler");
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
