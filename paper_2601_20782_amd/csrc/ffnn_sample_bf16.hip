// Register-resident dense-network sampler kernels with bf16 operands.
#include "ffnn_sample_inst.h"

namespace nqs {

bool ffnn_reg_sample_launch_bf16(int ke, bool trace, bool perchain, const FfnnSampleArgs &A, int blocks, size_t lds,
                              hipStream_t s)
{
    return launch_sample_ke<__bf16, 32>(ke, trace, perchain, A, blocks, lds, s);
}

size_t ffnn_reg_sample_lds_bf16(int N, int ke, int m2p)
{
    return RegSampleLds<__bf16>::bytes(N, ke, m2p);
}

}  // namespace nqs
