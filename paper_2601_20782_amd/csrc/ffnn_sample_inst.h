// Instantiations of the register-resident dense-network sampler, one per number of
// 16-wide fragments of the first hidden layer (KE = 5 .. 32); included by one
// source file per 16-bit type so that the two compile in parallel.
#pragma once

#include "ffnn_reg.h"

namespace nqs {

template <typename T, int KE, bool PERCHAIN>
static void launch_sample_form(bool trace, const FfnnSampleArgs &A, int blocks, size_t lds, hipStream_t s)
{
    if (trace) {
        allow_lds(ffnn_sample_reg_kernel<T, KE, true, PERCHAIN>, lds);
        hipLaunchKernelGGL((ffnn_sample_reg_kernel<T, KE, true, PERCHAIN>), dim3(blocks), dim3(kRegThreads), lds, s, A);
    } else {
        allow_lds(ffnn_sample_reg_kernel<T, KE, false, PERCHAIN>, lds);
        hipLaunchKernelGGL((ffnn_sample_reg_kernel<T, KE, false, PERCHAIN>), dim3(blocks), dim3(kRegThreads), lds, s, A);
    }
}

template <typename T, int KE>
static bool launch_sample_ke(int ke, bool trace, bool perchain, const FfnnSampleArgs &A, int blocks, size_t lds,
                             hipStream_t s)
{
    if (ke == KE) {
        if (perchain) launch_sample_form<T, KE, true>(trace, A, blocks, lds, s);
        else launch_sample_form<T, KE, false>(trace, A, blocks, lds, s);
        return true;
    }
    if constexpr (KE > 5) return launch_sample_ke<T, KE - 1>(ke, trace, perchain, A, blocks, lds, s);
    else return false;
}

}  // namespace nqs
