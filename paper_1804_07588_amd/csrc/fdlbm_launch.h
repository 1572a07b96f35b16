// Host-callable launchers of the step and observe kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "fdlbm_device.h"

namespace fdlbm {

enum { K_WALL_ID = 0, K_MOMENTS_ID = 1, K_COLLIDE_ID = 2, K_SOLID_ID = 3, K_NUM = 4 };

struct LaunchInfo {
  hipStream_t stream;
  int n_solid;
  hipEvent_t *events;  // 2 per kernel id (start, stop) or null
  bool recorded[K_NUM];  // set by the launcher for the ids it recorded
};

// one time step on lattice D: wall, moments, collide (with inlet/outlet),
// solid; real = arithmetic type, PT = population storage type
template <typename real, typename PT, int D>
hipError_t step_lat(const Params<real> &p, const Bufs<real, PT> &b, int cur, LaunchInfo &li);

// observables: writes (ns + 9) doubles per block into b.partials
template <typename real, typename PT, int D>
hipError_t observe_lat(const Params<real> &p, const Bufs<real, PT> &b, int cur, int blocks,
                       hipStream_t st);

// residual of the steady-state test: 8 doubles per block into b.partials
template <typename real, typename PT, int D>
hipError_t residual_lat(const Params<real> &p, const Bufs<real, PT> &b, int cur, int blocks,
                        hipStream_t st);

template <typename real, typename PT>
inline hipError_t launch_residual(int D, const Params<real> &p, const Bufs<real, PT> &b, int cur,
                                  int blocks, hipStream_t st) {
  return D == 2 ? residual_lat<real, PT, 2>(p, b, cur, blocks, st)
                : residual_lat<real, PT, 3>(p, b, cur, blocks, st);
}

template <typename real, typename PT>
inline hipError_t launch_step(int D, const Params<real> &p, const Bufs<real, PT> &b, int cur,
                              LaunchInfo &li) {
  return D == 2 ? step_lat<real, PT, 2>(p, b, cur, li) : step_lat<real, PT, 3>(p, b, cur, li);
}

template <typename real, typename PT>
inline hipError_t launch_observe(int D, const Params<real> &p, const Bufs<real, PT> &b, int cur,
                                 int blocks, hipStream_t st) {
  return D == 2 ? observe_lat<real, PT, 2>(p, b, cur, blocks, st)
                : observe_lat<real, PT, 3>(p, b, cur, blocks, st);
}

}  // namespace fdlbm
