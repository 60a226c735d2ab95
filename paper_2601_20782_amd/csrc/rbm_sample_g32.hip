// RBM sampler instantiations for 32 lanes per chain.
#include "rbm_sampler.h"

namespace nqs {

nqs_status rbm_sample_launch_g32(const RbmSampleArgs &A, const RbmLaunch &L, hipStream_t s)
{
    switch (L.K) {
    case 1: launch_rbm_sample_gk<32, 1>(A, L, s); break;
    case 2: launch_rbm_sample_gk<32, 2>(A, L, s); break;
    case 3: launch_rbm_sample_gk<32, 3>(A, L, s); break;
    case 4: launch_rbm_sample_gk<32, 4>(A, L, s); break;
    case 5: launch_rbm_sample_gk<32, 5>(A, L, s); break;
    case 6: launch_rbm_sample_gk<32, 6>(A, L, s); break;
    case 7: launch_rbm_sample_gk<32, 7>(A, L, s); break;
    case 8: launch_rbm_sample_gk<32, 8>(A, L, s); break;
    case 9: launch_rbm_sample_gk<32, 9>(A, L, s); break;
    case 10: launch_rbm_sample_gk<32, 10>(A, L, s); break;
    case 11: launch_rbm_sample_gk<32, 11>(A, L, s); break;
    case 12: launch_rbm_sample_gk<32, 12>(A, L, s); break;
    case 13: launch_rbm_sample_gk<32, 13>(A, L, s); break;
    case 14: launch_rbm_sample_gk<32, 14>(A, L, s); break;
    case 15: launch_rbm_sample_gk<32, 15>(A, L, s); break;
    case 16: launch_rbm_sample_gk<32, 16>(A, L, s); break;
    default: return set_error(NQS_EUNSUPPORTED, "hidden width too large for 32 lanes per chain");
    }
    NQS_HIP_TRY(hipGetLastError());
    return NQS_OK;
}

}  // namespace nqs
