// Register-resident local-energy kernels with bf16 operands.
#include "ffnn_eloc_inst.h"

namespace nqs {

bool ffnn_reg_eloc_launch_bf16(int ke, const FfnnElocArgs &A, int G, int blocks, size_t lds, hipStream_t s)
{
    return launch_eloc_ke<__bf16, 32>(ke, A, G, blocks, lds, s);
}

size_t ffnn_reg_eloc_lds_bf16(int N, int ke, int m2p, int G)
{
    return reg_eloc_lds_bytes<__bf16>(N, ke, m2p, G);
}

}  // namespace nqs
