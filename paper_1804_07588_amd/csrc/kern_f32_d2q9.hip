// Kernel instantiations: float storage and arithmetic on the D2Q9 lattice.
#define FDLBM_NS_CASES FDLBM_CASE(1) FDLBM_CASE(2) FDLBM_CASE(3) FDLBM_CASE(4) FDLBM_CASE(5) FDLBM_CASE(6)
#include "fdlbm_kernels_impl.h"

namespace fdlbm {
template hipError_t step_lat<float, float, 2>(const Params<float> &, const Bufs<float, float> &, int,
                                          LaunchInfo &);
template hipError_t observe_lat<float, float, 2>(const Params<float> &, const Bufs<float, float> &, int,
                                             int, hipStream_t);
template hipError_t residual_lat<float, float, 2>(const Params<float> &, const Bufs<float, float> &, int, int,
                                           hipStream_t);
template hipError_t batch_step_lat<float, float, 2>(int, const BatchLaunch &, int);
}  // namespace fdlbm
