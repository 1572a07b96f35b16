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
  // optional second stream: the wall and solid kernels run there, beside the
  // moments and collision kernels on `stream` (null: one stream)
  hipStream_t side;
  hipEvent_t ev_fork, ev_wall, ev_solid;
};

// Batched launches (many samples per launch): per launch kind, a device work
// list of (sample, logical block) pairs, its length in device memory (read by
// the kernels, so a captured graph follows later edits of the list), the
// largest length it may take (0: the launch is skipped) and the persistent
// grid (a multiple of 8 workgroups).
enum { BL_WALL_FAST = 0, BL_WALL_SLOW, BL_GAS_FAST, BL_GAS_SLOW, BL_COLLIDE, BL_SOLID, BL_NUM };
struct BatchLaunch {
  const void *params;  // Params<real>[n_samples], device
  const void *bufs;    // Bufs<real, PT>[n_samples], device
  const int2 *items[BL_NUM];
  const int *count;    // BL_NUM ints, device
  int max_items[BL_NUM];
  int grid[BL_NUM];
  hipStream_t stream;
  // optional second stream for the wall and solid launches (null: one stream)
  hipStream_t side;
  hipEvent_t ev_fork, ev_wall, ev_solid;
  // wall variants shared by every sample: half-way wall, several reactions;
  // eq48: the Eq.(48) solid coupling (the solid step follows the moments);
  // cn_iters: 0 for the forward-Euler solid, else the largest sample's
  // number of Crank-Nicolson Jacobi sweeps
  int halfway, multi, eq48, cn_iters;
};

template <typename real, typename PT, int D>
hipError_t batch_step_lat(int ns, const BatchLaunch &bl, int cur);

template <typename real, typename PT>
inline hipError_t launch_batch_step(int D, int ns, const BatchLaunch &bl, int cur) {
  return D == 2 ? batch_step_lat<real, PT, 2>(ns, bl, cur) : batch_step_lat<real, PT, 3>(ns, bl, cur);
}

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
