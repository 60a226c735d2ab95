// Dense-network (FFNN) kernels: exchange-move sampler, Heisenberg local energies, backward.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace nqs {

nqs_status ffnn_build_copy(nqs_model *, int, hipStream_t)
{
    return set_error(NQS_EUNSUPPORTED, "dense networks are not built yet");
}
nqs_status ffnn_sample(nqs_model *, const nqs_sample_cfg &, int8_t *, int8_t *, float *, uint64_t *, const nqs_trace *,
                       hipStream_t)
{
    return set_error(NQS_EUNSUPPORTED, "dense networks are not built yet");
}
nqs_status ffnn_local_energy(nqs_model *, const nqs_ham_desc &, const int8_t *, int64_t, int, double *, hipStream_t)
{
    return set_error(NQS_EUNSUPPORTED, "dense networks are not built yet");
}
nqs_status ffnn_logpsi_grad(nqs_model *, const int8_t *, int64_t, float *, float *, const float *, float *, hipStream_t)
{
    return set_error(NQS_EUNSUPPORTED, "dense networks are not built yet");
}

}  // namespace nqs
