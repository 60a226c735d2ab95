// Register-resident local-energy kernels with f16 operands.
#include "ffnn_eloc_inst.h"

namespace nqs {

bool ffnn_reg_eloc_launch_f16(int ke, const FfnnElocArgs &A, int G, int blocks, size_t lds, hipStream_t s)
{
    return launch_eloc_ke<_Float16, 32>(ke, A, G, blocks, lds, s);
}

size_t ffnn_reg_eloc_lds_f16(int N, int ke, int m2p, int G)
{
    return reg_eloc_lds_bytes<_Float16>(N, ke, m2p, G);
}

}  // namespace nqs
