// Instantiations of the register-resident local-energy kernel, one per number of
// 16-wide fragments of the first hidden layer (KE = 5 .. 32); included by one
// source file per 16-bit type so that the two compile in parallel.
#pragma once

#include "ffnn_reg.h"

namespace nqs {

template <typename T, int KE>
static bool launch_eloc_ke(int ke, const FfnnElocArgs &A, int G, int blocks, size_t lds, hipStream_t s)
{
    if (ke == KE) {
        allow_lds(ffnn_eloc_reg_kernel<T, KE>, lds);
        hipLaunchKernelGGL((ffnn_eloc_reg_kernel<T, KE>), dim3(blocks), dim3(kRegThreads), lds, s, A, G);
        return true;
    }
    if constexpr (KE > 5) return launch_eloc_ke<T, KE - 1>(ke, A, G, blocks, lds, s);
    else return false;
}

}  // namespace nqs
