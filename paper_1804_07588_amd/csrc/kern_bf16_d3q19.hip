// Kernel instantiations: BF16 population storage (deviations), float arithmetic on the D3Q19 lattice.
#define FDLBM_NS_CASES FDLBM_CASE(1) FDLBM_CASE(2) FDLBM_CASE(3) FDLBM_CASE(4) FDLBM_CASE(5) FDLBM_CASE(6)
#include "fdlbm_kernels_impl.h"

namespace fdlbm {
template hipError_t step_lat<float, __bf16, 3>(const Params<float> &, const Bufs<float, __bf16> &, int,
                                          LaunchInfo &);
template hipError_t observe_lat<float, __bf16, 3>(const Params<float> &, const Bufs<float, __bf16> &, int,
                                             int, hipStream_t);
template hipError_t residual_lat<float, __bf16, 3>(const Params<float> &, const Bufs<float, __bf16> &, int, int,
                                           hipStream_t);
template hipError_t batch_step_lat<float, __bf16, 3>(int, const BatchLaunch &, int);
}  // namespace fdlbm
