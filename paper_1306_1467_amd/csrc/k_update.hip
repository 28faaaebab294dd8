// Per-round update kernel of one job: the second level of the argmin, split
// rank, threshold, beta and alpha (Section 2.3 steps 3-4), and the weight
// update w_i <- w_i beta^(1 - e_i) with per-workgroup partial sums for the
// next normalisation.
#include "update_core.h"

namespace vjb {

template <int PREC>
__global__ __launch_bounds__(kUpdWg) void k_update(JobDev jd, int n_wg) {
    update_body<PREC>(jd, jd.wgb, n_wg, blockIdx.x);
}

int update_launch(const JobDev& jd, int n_wg, hipStream_t s) {
    const void* k;
    switch (jd.precision) {
    case BOOST_PREC_FP32: k = (const void*)k_update<BOOST_PREC_FP32>; break;
    case BOOST_PREC_FP32_KAHAN: k = (const void*)k_update<BOOST_PREC_FP32_KAHAN>; break;
    case BOOST_PREC_FP64: k = (const void*)k_update<BOOST_PREC_FP64>; break;
    default: k = (const void*)k_update<BOOST_PREC_FP32_WIDE>; break;
    }
    JobDev a = jd;
    void* args[] = {(void*)&a, (void*)&n_wg};
    VJB_HIP(hipLaunchKernel(k, dim3((unsigned)jd.n_part), dim3(kUpdWg), args, 0, s));
    return BOOST_OK;
}

}  // namespace vjb
