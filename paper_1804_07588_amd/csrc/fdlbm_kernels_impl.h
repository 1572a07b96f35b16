// HIP kernels (gfx950) of the coupled FD-LBM time step.
//
// Per step (k_wall then k_solid on a second stream beside k_moments then
// k_collide, ordered by events; or all four in sequence on one stream):
//   k_wall     reactive diffusive wall at every wall node: streaming of the
//              populations arriving from the gas, wall densities and the
//              thermalised emission (Eq.(37)-(42), (50))
//   k_moments  streaming into every gas node (Eq.(33)-(36)), stored for the
//              collision, and everything local: moments, transport, U^c,
//              species momenta of f (Eq.(3), (5), (7)-(8), (11), (14)-(17), (25))
//   k_collide  correction sources of all species from the
//              node's and its face neighbours' moments, the temperatures of f
//              and of the auxiliary state, equilibria and the trapezoidal
//              collision (Eq.(4), (6), (12)-(13), (19)-(21), (24)); writes the
//              inlet/outlet planes directly
//   k_solid    heat step in the solid on an LDS tile with the wall-node
//              interface source (Eq.(45)-(48)): forward Euler, or
//              Crank-Nicolson solved by Jacobi sweeps (k_solid_pass)
//
// Storage is per SLOT (gas nodes in processing order, then wall nodes).
// Populations are records of the NS species per (direction, slot),
// [((i*nsl + slot)*NS + j]: a tap of one direction is one contiguous record
// load that serves every species, and a wavefront of consecutive slots reads
// consecutive records.  Only the moments kernel gathers taps; it stores the
// streamed records in slot order, so the collision reads them as contiguous
// records (a gather costs several times a coalesced load on this GPU).
// Populations that only the next step reads (post-collision and
// wall-emitted) are written with non-temporal stores.
#pragma once
#include <type_traits>

#include "fdlbm_device.h"
#include "fdlbm_launch.h"

namespace fdlbm {

// periodic wrap of v in [-3, n + 2] (any n >= 1), branch-free
__device__ inline int wrapc(int v, int n) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    v = v < 0 ? v + n : v;
    v = v >= n ? v - n : v;
  }
  return v;
}

// Blocks are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous run of logical blocks, so slot neighbours (adjacent rows) are
// processed by one XCD close in time and share its L2.  Launch xcd_grid(nb)
// blocks; logical ids >= nb do nothing.
constexpr int NXCD = 8;
__host__ __device__ inline int xcd_grid(int nb) { return ((nb + NXCD - 1) / NXCD) * NXCD; }
__device__ inline int xcd_block(int nb) {
  const int per = (nb + NXCD - 1) / NXCD;
  return (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
}
// The same runs walked from their ends: a kernel that reads what the previous
// kernel wrote in xcd_block order starts with the records written last, which
// are the likeliest to be still cached.
__device__ inline int xcd_block_reversed(int nb) {
  const int per = (nb + NXCD - 1) / NXCD;
  return (int)(blockIdx.x % NXCD) * per + (per - 1 - (int)(blockIdx.x / NXCD));
}

// Per-thread addressing: taps are node + k*stride(i) unless a periodic axis
// wraps within 3 nodes (FAST = the node list holds no such node).
template <int D>
struct Addr {
  int node, x, y, z, nx, ny, nz;
  template <typename real>
  __device__ Addr(int nd, const Params<real> &p) : node(nd), nx(p.nx), ny(p.ny), nz(p.nz) {
    x = nd % nx;
    const int r = nd / nx;
    y = r % ny;
    z = r / ny;
  }
  template <bool FAST>
  __device__ inline int at(int i, int k) const {
    if constexpr (FAST) {
      return node + k * (cvec<D>(i, 0) + nx * (cvec<D>(i, 1) + ny * cvec<D>(i, 2)));
    } else {
      const int xx = wrapc(x + k * cvec<D>(i, 0), nx);
      const int yy = wrapc(y + k * cvec<D>(i, 1), ny);
      const int zz = D == 3 ? wrapc(z + k * cvec<D>(i, 2), nz) : 0;
      return xx + nx * (yy + ny * zz);
    }
  }
  // face neighbour along axis a, direction d (+1/-1); -1 outside a closed axis
  template <typename real>
  __device__ inline int face(const Params<real> &p, int a, int d) const {
    int q[3] = {x, y, z};
    const int lim[3] = {nx, ny, nz};
    q[a] += d;
    if (q[a] < 0 || q[a] >= lim[a]) {
      if (!p.per[a]) return -1;
      q[a] = q[a] < 0 ? q[a] + lim[a] : q[a] - lim[a];
    }
    return q[0] + nx * (q[1] + ny * q[2]);
  }
};

// Streaming weights per species and stencil class, staged in LDS by every
// kernel that streams (taps beyond a class's count carry weight 0).
template <typename real>
struct WTab {
  real w[MAX_NS][8][3];
};

template <typename real, int NS>
__device__ inline void load_wtab(const Params<real> &p, WTab<real> &wt) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int c = 0; c < 7; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) wt.w[j][c][k] = p.wint[j][c][k];
  }
  __syncthreads();
}

// Tap offsets (units of e_i from the destination) of each stencil class,
// packed 3 bits each (offset + 3); a class with fewer than three taps
// repeats one of its taps with weight 0.
// class: 0 (-2,-1,0)  1 (-1,0,1)  2 (-1,-2,-3)  3 (-1,0,0)  4 (-2,-1,-1)
//        5 (-1,-1,-1) 6 (0,0,0)
__device__ constexpr uint64_t pack_offsets() {
  constexpr int off[7][3] = {{-2, -1, 0}, {-1, 0, 1}, {-1, -2, -3}, {-1, 0, 0},
                             {-2, -1, -1}, {-1, -1, -1}, {0, 0, 0}};
  uint64_t v = 0;
  for (int c = 0; c < 7; ++c)
    for (int k = 0; k < 3; ++k) v |= uint64_t(off[c][k] + 3) << (9 * c + 3 * k);
  return v;
}

// load base[idx] with a uniform base (SGPRs) and a 32-bit per-lane byte offset
template <typename T>
__device__ inline T ld(const T *__restrict__ base, int idx) {
  const uint32_t off = uint32_t(idx) * uint32_t(sizeof(T));
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T>
__device__ inline void st(T *__restrict__ base, int idx, T v) {
  const uint32_t off = uint32_t(idx) * uint32_t(sizeof(T));
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

// N consecutive values: record `rec` of an array of N-value records, moved as
// one contiguous access per lane (the compiler splits it into the widest
// loads and stores the element alignment allows).  64-bit byte offsets: the
// moment records (up to 192 bytes per slot) exceed 4 GiB on large domains.
template <typename real, int N>
struct Rec {
  real v[N];
};
template <typename real, int N>
__device__ inline Rec<real, N> ldrec(const real *__restrict__ base, int rec) {
  const size_t off = size_t(rec) * (N * sizeof(real));
  const real *p = reinterpret_cast<const real *>(reinterpret_cast<const char *>(base) + off);
  Rec<real, N> r;
  __builtin_memcpy(&r, p, sizeof r);
  return r;
}
template <typename real, int N>
__device__ inline void strec(real *__restrict__ base, int rec, const Rec<real, N> &r) {
  const size_t off = size_t(rec) * (N * sizeof(real));
  real *p = reinterpret_cast<real *>(reinterpret_cast<char *>(base) + off);
  __builtin_memcpy(p, &r, sizeof r);
}
// the first K values of record `rec` of an array of N-value records
template <typename real, int N, int K>
__device__ inline Rec<real, K> ldhead(const real *__restrict__ base, int rec) {
  const size_t off = size_t(rec) * (N * sizeof(real));
  const real *p = reinterpret_cast<const real *>(reinterpret_cast<const char *>(base) + off);
  Rec<real, K> r;
  __builtin_memcpy(&r, p, sizeof r);
  return r;
}

// Population records: RL = rec_len<PT>(NS) stored values per (direction,
// slot).  For a 16-bit storage type the record is moved as 4-byte words and
// holds relative deviations g / rho_ref_j - wlat_i; pop_load / pop_store
// convert to and from the populations themselves.
template <typename real, typename PT, int NS>
__device__ inline Rec<real, NS> pop_load_raw(const PT *__restrict__ Gi, int slot) {
  constexpr int RL = rec_len<PT>(NS);
  Rec<real, NS> r;
  if constexpr (narrow<PT>()) {
    const uint32_t off = uint32_t(slot) * uint32_t(RL * sizeof(PT));
    const uint32_t *p = reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(Gi) + off);
    Rec<uint32_t, RL / 2> w;
    __builtin_memcpy(&w, p, sizeof w);
    PT h[RL];
    __builtin_memcpy(h, &w, sizeof h);
#pragma unroll
    for (int j = 0; j < NS; ++j) r.v[j] = real(float(h[j]));
  } else {
    // 32-bit byte offset within one direction's array (the geometry set-up
    // rejects domains whose per-direction arrays would exceed 4 GiB)
    const uint32_t off = uint32_t(slot) * uint32_t(NS * sizeof(real));
    __builtin_memcpy(&r, reinterpret_cast<const char *>(Gi) + off, sizeof r);
  }
  return r;
}
// NW 4-byte words to a 4-byte aligned address with the non-temporal hint, in
// the widest vector stores that alignment allows
template <int NW>
__device__ inline void st_words_nt(uint32_t *__restrict__ p, const uint32_t *w) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4), aligned(4)));
  typedef uint32_t u3 __attribute__((ext_vector_type(3), aligned(4)));
  typedef uint32_t u2 __attribute__((ext_vector_type(2), aligned(4)));
  constexpr int N4 = NW / 4, R = NW % 4;
#pragma unroll
  for (int k = 0; k < N4; ++k) {
    const u4 x = {w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]};
    __builtin_nontemporal_store(x, reinterpret_cast<u4 *>(p + 4 * k));
  }
  if constexpr (R == 3) {
    const u3 x = {w[4 * N4], w[4 * N4 + 1], w[4 * N4 + 2]};
    __builtin_nontemporal_store(x, reinterpret_cast<u3 *>(p + 4 * N4));
  } else if constexpr (R == 2) {
    const u2 x = {w[4 * N4], w[4 * N4 + 1]};
    __builtin_nontemporal_store(x, reinterpret_cast<u2 *>(p + 4 * N4));
  } else if constexpr (R == 1) {
    __builtin_nontemporal_store(w[4 * N4], p + 4 * N4);
  }
}

// NT: a streaming (non-temporal) store, for populations that no kernel of
// the same step reads again (the post-collision and wall-emitted populations,
// read by the next step after the rest of this step's traffic)
template <typename real, typename PT, int NS, bool NT = false>
__device__ inline void pop_store_raw(PT *__restrict__ Gi, int slot, const Rec<real, NS> &v) {
  constexpr int RL = rec_len<PT>(NS);
  constexpr int NW = int(RL * sizeof(PT)) / 4;
  static_assert(RL * sizeof(PT) % 4 == 0, "records are whole 4-byte words");
  const uint32_t off = uint32_t(slot) * uint32_t(RL * sizeof(PT));
  uint32_t *p = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(Gi) + off);
  uint32_t w[NW];
  if constexpr (narrow<PT>()) {
    PT h[RL];
#pragma unroll
    for (int j = 0; j < RL; ++j) h[j] = j < NS ? PT(float(v.v[j])) : PT(0.0f);
    __builtin_memcpy(w, h, sizeof w);
  } else {
    __builtin_memcpy(w, &v, sizeof w);
  }
  if constexpr (NT) st_words_nt<NW>(p, w);
  else __builtin_memcpy(p, w, sizeof w);
}
// The 16-bit storage transform g = (d + w_i) rho_ref and its inverse, kept
// out of floating-point contraction: the compiler would otherwise fuse them
// with neighbouring arithmetic differently in different kernels, and the
// batched and single-domain launches would round stored values differently.
template <typename real>
__device__ inline real dev_decode(real d, real w, real rho_ref) {
#pragma clang fp contract(off)
  return (d + w) * rho_ref;
}
template <typename real>
__device__ inline real dev_encode(real g, real inv_rho_ref, real w) {
#pragma clang fp contract(off)
  return g * inv_rho_ref - w;
}
template <typename real, typename PT, int D, int NS>
__device__ inline Rec<real, NS> pop_load(const Params<real> &p, const PT *__restrict__ Gi, int slot, int i) {
  Rec<real, NS> r = pop_load_raw<real, PT, NS>(Gi, slot);
  if constexpr (narrow<PT>()) {
#pragma unroll
    for (int j = 0; j < NS; ++j) r.v[j] = dev_decode(r.v[j], real(wlat<D>(i)), p.rho_ref[j]);
  }
  return r;
}
template <typename real, typename PT, int D, int NS, bool NT = false>
__device__ inline void pop_store(const Params<real> &p, PT *__restrict__ Gi, int slot, int i, Rec<real, NS> v) {
  if constexpr (narrow<PT>()) {
#pragma unroll
    for (int j = 0; j < NS; ++j) v.v[j] = dev_encode(v.v[j], p.inv_rho_ref[j], real(wlat<D>(i)));
  }
  pop_store_raw<real, PT, NS, NT>(Gi, slot, v);
}
// store into the next step's buffer (streaming)
template <typename real, typename PT, int D, int NS>
__device__ inline void pop_store_next(const Params<real> &p, PT *__restrict__ Gi, int slot, int i,
                                      const Rec<real, NS> &v) {
  pop_store<real, PT, D, NS, true>(p, Gi, slot, i, v);
}

// Slots of the three taps of direction i for stencil class cls (0..6) around
// the node of ad, Eq.(33)-(36).
struct TapSlots {
  int s[3];
};
template <bool FAST, int D, typename BF>
__device__ inline TapSlots tap_slots(const BF &b, const Addr<D> &ad, int i, int cls) {
  constexpr uint64_t OFF = pack_offsets();
  const int sh = 9 * cls;
  TapSlots t;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int o = int((OFF >> (sh + 3 * k)) & 7u) - 3;
    t.s[k] = ld(b.slot_of, ad.template at<FAST>(i, o));
  }
  return t;
}

// Pre-collision populations of all NS species in direction i (array Gi, the
// records of direction i): the interpolant through the class's taps at each
// species' shift.  An on-lattice species (c_j = 1) has weights exactly one 1
// and two 0s, so it gets the upstream value unrounded.
template <typename real, typename PT, int D, int NS>
__device__ inline Rec<real, NS> stream_rec(const Params<real> &p, const PT *__restrict__ Gi, const TapSlots &t,
                                           const WTab<real> &wt, int cls, int i) {
  const Rec<real, NS> r0 = pop_load_raw<real, PT, NS>(Gi, t.s[0]);
  const Rec<real, NS> r1 = pop_load_raw<real, PT, NS>(Gi, t.s[1]);
  const Rec<real, NS> r2 = pop_load_raw<real, PT, NS>(Gi, t.s[2]);
  Rec<real, NS> g;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    g.v[j] = wt.w[j][cls][0] * r0.v[j] + wt.w[j][cls][1] * r1.v[j] + wt.w[j][cls][2] * r2.v[j];
    // the weights sum to one: deviations interpolate like the populations
    if constexpr (narrow<PT>()) g.v[j] = dev_decode(g.v[j], real(wlat<D>(i)), p.rho_ref[j]);
  }
  return g;
}

// Gas destinations: a gas node emits along every direction, so the class
// search never reaches class 2 (it needs x - e and x - 2e, which would make
// class 0 valid).  Every other class can then list its taps as (two looked-up
// nodes, the node itself), so one of the three taps is the destination's own
// slot: no slot lookup, and a coalesced record load across the wavefront.
// Offsets of the two looked-up taps per class, and where each original tap
// weight goes (original tap k -> new position, -1: the weight is 0 and the
// original tap is dropped).
__device__ constexpr int gas_off(int cls, int k) {
  constexpr int off[7][2] = {{-2, -1}, {-1, 1}, {-1, -2}, {-1, -1}, {-2, -1}, {-1, -1}, {0, 0}};
  return off[cls][k];
}
template <typename real, int NS>
__device__ inline void load_wtab_gas(const Params<real> &p, WTab<real> &wt) {
  // new tap order per class: (looked-up 0, looked-up 1, own node)
  constexpr int src[7][3] = {{0, 1, 2}, {0, 2, 1}, {0, 1, 2}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1}, {-1, -1, 0}};
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int c = 0; c < 7; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) wt.w[j][c][k] = src[c][k] < 0 ? real(0) : p.wint[j][c][src[c][k]];
  }
  __syncthreads();
}
template <bool FAST, int D, typename BF>
__device__ inline TapSlots gas_tap_slots(const BF &b, const Addr<D> &ad, int i, int cls, int t) {
  constexpr uint64_t OFF = [] {
    uint64_t v = 0;
    for (int c = 0; c < 7; ++c)
      for (int k = 0; k < 2; ++k) v |= uint64_t(gas_off(c, k) + 3) << (6 * c + 3 * k);
    return v;
  }();
  const int sh = 6 * cls;
  TapSlots ts;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int o = int((OFF >> (sh + 3 * k)) & 7u) - 3;
    ts.s[k] = ld(b.slot_of, ad.template at<FAST>(i, o));
  }
  ts.s[2] = t;
  return ts;
}

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, typename F>
__device__ inline void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ inline int cls_at(uint64_t w, int i) { return int((w >> (3 * (i - 1))) & 7u); }

// block-wide FP64 sum in a fixed order (deterministic); result in thread 0
__device__ inline double block_sum(double v) {
  __shared__ double sh[BLOCK];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

template <typename real>
__device__ inline real tiny() {
  return sizeof(real) == 4 ? real(1e-30f) : real(1e-300);
}

template <typename real>
__device__ inline real ipow(real x, int k) {
  real r = real(1);
  for (int q = 0; q < k; ++q) r *= x;
  return r;
}

// ===========================================================================
// k_wall: the reactive diffusive wall, one thread per wall node
// ===========================================================================
// Several surface reactions at one wall node (the flux boundary condition
// takes any source; with several reactions S_j sums theirs).  A_j arriving
// mass, Zj_j emission weights, area the rate factor, rw_j in: A_j / Zj_j.
// The fixed point updates the species some reaction consumes with a
// positive order, each with its own consumption implicit and its production
// at the current densities; then the rates at the converged densities and
// the wall densities from the exact mass balance.  r: the summed rates
// (moles per step), q: the reaction heat sum_k -dH_k r_k (Eq.(42)).
template <typename real, int NS>
__device__ inline void several_reactions(const Params<real> &p, const real *__restrict__ rxt, const real (&A)[NS],
                                         const real (&Zj)[NS], real area, real Tw, real (&rw)[NS], real &r,
                                         real &q) {
  real kk[MAXR];
  unsigned upd = 0;
#pragma unroll
  for (int k = 0; k < MAXR; ++k) {
    kk[k] = real(0);
    if (k < p.n_rx) {
      const real *t = rxt + k * RXS;
      kk[k] = area * t[RX_K0] * exp(t[RX_EA] * (real(1) - t[RX_TREF] / Tw));
#pragma unroll
      for (int j = 0; j < NS; ++j)
        if (t[RX_NU + j] < real(0) && t[RX_ORD + j] > real(0)) upd |= 1u << j;
    }
  }
  // rate of reaction k at rw, or (lower >= 0) divided by C_lower: that
  // species' power lowered by one (lower has a positive order in k)
  auto rate = [&](int k, int lower) {
    const real *t = rxt + k * RXS;
    real v = kk[k];
#pragma unroll
    for (int m = 0; m < NS; ++m) v *= ipow(rw[m] * p.invM[m], (int)t[RX_ORD + m] - (m == lower ? 1 : 0));
    return v;
  };
  for (int it = 0; it < p.max_iter; ++it) {
    real rk[MAXR];
#pragma unroll
    for (int k = 0; k < MAXR; ++k) rk[k] = k < p.n_rx ? rate(k, -1) : real(0);
    real nw[NS], dmax = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      nw[j] = rw[j];
      if ((upd >> j) & 1u) {
        real num = 0, den = 0;
#pragma unroll
        for (int k = 0; k < MAXR; ++k) {
          if (k >= p.n_rx) continue;
          const real *t = rxt + k * RXS;
          const real nu = t[RX_NU + j];
          if (nu < real(0) && t[RX_ORD + j] > real(0)) den += nu * p.srcf[j] * rate(k, j);
          else if (nu != real(0)) num += nu * p.M[j] * p.srcf[j] * rk[k];
        }
        nw[j] = (A[j] + num) / (Zj[j] - den);
      }
      dmax = fmax(dmax, fabs(nw[j] - rw[j]) / fmax(fabs(nw[j]), tiny<real>()));
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) rw[j] = nw[j];
    if (dmax <= p.tol) break;
  }
  real rk[MAXR];
#pragma unroll
  for (int k = 0; k < MAXR; ++k) rk[k] = k < p.n_rx ? rate(k, -1) : real(0);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    real src = 0;
#pragma unroll
    for (int k = 0; k < MAXR; ++k)
      if (k < p.n_rx) src += rxt[k * RXS + RX_NU + j] * p.M[j] * p.srcf[j] * rk[k];
    rw[j] = (A[j] + src) / Zj[j];
  }
  r = 0;
  q = 0;
#pragma unroll
  for (int k = 0; k < MAXR; ++k)
    if (k < p.n_rx) {
      r += rk[k];
      q += -rxt[k * RXS + RX_DH] * rk[k];
    }
}

// what a wall node hands to its block's sums: the moles reacted and (several
// reactions) the reaction heat
struct WallOut {
  double r, q;
};

// Half-way wall (Sec. 4.3; the interpolation step taken linear): along link i
// into gas node x the wall node thermalises at the state whose linear
// interpolant with x takes the wall's values at the link's midpoint,
// velocity -u(x) and temperature 2 T_w - T(x), read from x's moment record
// of the previous step.  Weights f^eq_ji(1, -u(x), 2 T_w - T(x)) of every
// species for the compile-time direction I.
template <int I, bool FAST, typename real, int D, int NS, typename BF>
__device__ inline void halfway_weights(const Params<real> &p, const BF &b, const Addr<D> &ad, real Tw,
                                       real (&f)[NS]) {
  constexpr int NR = fr_count(D, NS);
  const int xs = ld(b.slot_of, ad.template at<FAST>(I, 1));
  const Rec<real, D + 1> h = ldhead<real, NR, D + 1>(b.FR, xs);
  real ul[3] = {real(0), real(0), real(0)};
#pragma unroll
  for (int a = 0; a < D; ++a) ul[a] = -h.v[fr_u(a)];
  const real Tl = real(2) * Tw - h.v[fr_T(D)];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    real e[lat_q<D>()];
    equilibrium<real, D>(real(1), p.sqM[j], ul, Tl, e);
    f[j] = e[I];
  }
}

// HALF: the half-way wall; MULTI: several surface reactions (separate
// instantiations, so that the common kernel keeps its register budget)
template <bool FAST, bool HALF, bool MULTI, typename real, typename PT, int D, int NS>
__device__ inline WallOut wall_node(const Params<real> &p, const Bufs<real, PT> &b, int cur,
                                    const WTab<real> &wtab, const int wi) {
  constexpr int Q = lat_q<D>();
  constexpr int NR = fr_count(D, NS);
  const int slot = p.n_gas + wi;
  const int w = (int)b.wall_list[wi];
  const Addr<D> ad(w, p);
  const uint64_t cw = b.scls[slot];
  const uint32_t em = b.wem[wi];
  constexpr int RL = rec_len<PT>(NS);
  const PT *__restrict__ G = b.G[cur];
  PT *__restrict__ Gn = b.G[cur ^ 1];
  const int nsl = p.nsl;
  const real Tw = p.wall_mode == 1 ? p.T_iso : b.Ts[cur][w];
  real wt[Q];
  const real u0[3] = {0, 0, 0};
  equilibrium<real, D>(real(1), real(1), u0, Tw, wt);
  // Z: thermalised emission weight summed over the links into the gas
  real Z = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (em & (1u << i)) Z += wt[i];
  // the emission weight of each species: Z, or for the half-way wall the
  // sum of its per-link weights
  real Zj[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) Zj[j] = HALF ? real(0) : Z;
  if constexpr (HALF) {
    static_for<1, Q>([&](auto I) {
      if (em & (1u << I.value)) {
        real f[NS];
        halfway_weights<I.value, FAST, real, D, NS>(p, b, ad, Tw, f);
#pragma unroll
        for (int j = 0; j < NS; ++j) Zj[j] += f[j];
      }
    });
  }
  // A_j: mass arriving from the gas (incoming links), with its energy
  real A[NS], Ej[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) A[j] = Ej[j] = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int cls = cls_at(cw, i);
    if (cls == CLS_NONE) continue;  // direction i does not arrive from the gas
    const Rec<real, NS> g =
        stream_rec<real, PT, D, NS>(p, G + (size_t)i * nsl * RL, tap_slots<FAST>(b, ad, i, cls), wtab, cls, i);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      A[j] += g.v[j];
      Ej[j] += real(cnorm2<D>(i)) * g.v[j];
    }
  }
  real Ein = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) Ein += p.cj2[j] * Ej[j];
  // wall densities: rho_w,j Z = A_j + nu_j M_j r s_j (Eq.(41) with Eq.(50);
  // s_j = 1, or 1 / c_j for a stoichiometric mass flux out of the wall);
  // fixed point started at the non-reactive density, each reactant's own
  // concentration treated implicitly
  real rw[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) rw[j] = A[j] / Zj[j];
  // rate constant at T_w (Eq.(50) with the Arrhenius factor); one reaction
  // term per wall node, corners included (Sec. 4.3), or, as an option, per
  // unit wetted area: the node's rest emission weight over its links into
  // the gas relative to a plane wall's T_w / 2 (Z itself: the rest weights)
  const real area = p.rate_area ? Z / (real(0.5) * Tw) : real(1);
  real r, q = 0;
  if constexpr (MULTI) {
    several_reactions<real, NS>(p, b.rxt, A, Zj, area, Tw, rw, r, q);
  } else {
    const real keff = area * p.k0 * exp(p.ea * (real(1) - p.T_ref_rxn / Tw));
    for (int it = 0; it < p.max_iter; ++it) {
      real nw[NS], dmax = 0;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        nw[j] = rw[j];
        if (p.nu[j] < real(0) && p.order[j] > 0) {
          real R = keff;
#pragma unroll
          for (int m = 0; m < NS; ++m) R *= ipow(rw[m] * p.invM[m], p.order[m] - (m == j ? 1 : 0));
          nw[j] = A[j] / (Zj[j] - p.nu[j] * p.srcf[j] * R);
        }
        const real d = fabs(nw[j] - rw[j]) / fmax(fabs(nw[j]), tiny<real>());
        dmax = fmax(dmax, d);
      }
#pragma unroll
      for (int j = 0; j < NS; ++j) rw[j] = nw[j];
      if (dmax <= p.tol) break;
    }
    r = keff;
#pragma unroll
    for (int m = 0; m < NS; ++m) r *= ipow(rw[m] * p.invM[m], p.order[m]);
    if constexpr (HALF) {
#pragma unroll
      for (int j = 0; j < NS; ++j) rw[j] = (A[j] + p.nu[j] * p.M[j] * p.srcf[j] * r) / Zj[j];
    } else {
      const real invZ = real(1) / Z;
#pragma unroll
      for (int j = 0; j < NS; ++j) rw[j] = (A[j] + p.nu[j] * p.M[j] * p.srcf[j] * r) * invZ;
    }
  }
  // emission: rho_w,j f^eq_i(1, 0, T_w) on the links into the gas (half-way:
  // the link's own weights, computed again)
  real Eout = 0;
  static_for<1, Q>([&](auto I) {
    constexpr int i = I.value;
    if (!(em & (1u << i))) return;
    real f[NS];
    if constexpr (HALF) halfway_weights<i, FAST, real, D, NS>(p, b, ad, Tw, f);
    Rec<real, NS> W;
    real Ei = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      W.v[j] = rw[j] * (HALF ? f[j] : wt[i]);
      Ei += p.cj2[j] * W.v[j];
    }
    pop_store_next<real, PT, D, NS>(p, Gn + (size_t)i * nsl * RL, slot, i, W);
    Eout += real(cnorm2<D>(i)) * Ei;
  });
  // wall state seen by the neighbours' gradient stencils
  Rec<real, NR> fr;
#pragma unroll
  for (int a = 0; a < D; ++a) fr.v[fr_u(a)] = real(0);
  fr.v[fr_T(D)] = Tw;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    fr.v[fr_rho(D, j)] = rw[j];
    fr.v[fr_tau1(D, j)] = real(0);
  }
  strec<real, NR>(b.FR, slot, fr);
  b.wall_r[w] = r;
  if constexpr (MULTI) b.wall_q[w] = q;
  b.wall_dE[w] = real(0.5) * (Eout - Ein);
  return WallOut{(double)r, (double)q};
}

// FAST: the node list holds only nodes whose taps never wrap a periodic axis.
// One block of wall nodes (logical block lb of the list).
template <bool FAST, bool HALF, bool MULTI, typename real, typename PT, int D, int NS>
__device__ __forceinline__ void wall_block(const Params<real> &p, const Bufs<real, PT> &b, int cur,
                                           const WTab<real> &wtab, int lb) {
  const int first = FAST ? 0 : p.n_wall_fast, count = FAST ? p.n_wall_fast : p.n_wall - p.n_wall_fast;
  const int t = lb * BLOCK + threadIdx.x;
  WallOut o{0.0, 0.0};
  if (t < count) o = wall_node<FAST, HALF, MULTI, real, PT, D, NS>(p, b, cur, wtab, first + t);
  const int slot = lb + (FAST ? 0 : p.slot_off_wall);
  const double s = block_sum(o.r);
  if (threadIdx.x == 0) b.acc_moles[slot] += s;
  if constexpr (MULTI) {
    const double sq = block_sum(o.q);
    if (threadIdx.x == 0) b.acc_heat[slot] += sq;
  }
}
template <bool FAST, bool HALF, bool MULTI, typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK) k_wall(Params<real> p, Bufs<real, PT> b, int cur) {
  __shared__ WTab<real> wtab;
  load_wtab<real, NS>(p, wtab);
  const int count = FAST ? p.n_wall_fast : p.n_wall - p.n_wall_fast;
  const int nb = (count + BLOCK - 1) / BLOCK, lb = xcd_block(nb);
  if (lb >= nb) return;  // whole block: no barrier follows for it
  wall_block<FAST, HALF, MULTI, real, PT, D, NS>(p, b, cur, wtab, lb);
}

// ===========================================================================
// k_moments: streaming into every gas node (stored for the collision), the
// moments of the streamed populations and every local quantity of the node
// (Eq.(3), (5), (7)-(8), (11), (14)-(17), (25)), one thread per node.
// ===========================================================================
// collision integral at reduced temperature ts from a table on a uniform grid
// (linear interpolation, constant beyond the ends)
template <typename real>
__device__ inline real lj_omega(const Params<real> &p, const real *tab, real ts) {
  const real f = (ts - p.lj_t0) * p.lj_idt;
  if (!(f > real(0))) return tab[0];
  if (f >= real(p.lj_n - 1)) return tab[p.lj_n - 1];
  const int i = (int)f;
  const real w = f - real(i);
  return (real(1) - w) * tab[i] + w * tab[i + 1];
}

// one gas node (slot t) of the streaming-and-moments pass
template <bool FAST, typename real, typename PT, int D, int NS>
__device__ __forceinline__ void moments_node(const Params<real> &p, const Bufs<real, PT> &b, int cur,
                                             const WTab<real> &wtab, int t) {
  constexpr int Q = lat_q<D>();
  constexpr int NR = fr_count(D, NS), NX = fx_count(D, NS);
  const int node = (int)b.gas_list[t];
  const Addr<D> ad(node, p);
  const uint64_t cw = b.scls[t];
  constexpr int RL = rec_len<PT>(NS);
  const PT *__restrict__ G = b.G[cur];
  const int nsl = p.nsl;
  real rho[NS], Jg[NS][D], Es[NS];
  {
    const Rec<real, NS> g0 = pop_load<real, PT, D, NS>(p, G, t, 0);  // rest population: not streamed
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      rho[j] = g0.v[j];
      Es[j] = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) Jg[j][a] = 0;
    }
  }
  static_for<1, Q>([&](auto ic_) __attribute__((always_inline)) {
    constexpr int i = decltype(ic_)::value;
    const int cls = cls_at(cw, i);
    const Rec<real, NS> g = stream_rec<real, PT, D, NS>(p, G + (size_t)i * nsl * RL,
                                                     gas_tap_slots<FAST>(b, ad, i, cls, t), wtab, cls, i);
    // streaming store: the collision reads it in its own launch, after more
    // than the L2 holds has passed (measured 3 % faster than a cached store
    // here, 1 % slower to read back)
    pop_store<real, PT, D, NS, true>(p, b.Gs + (size_t)i * nsl * RL, t, i, g);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      rho[j] += g.v[j];
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (cvec<D>(i, a) != 0) Jg[j][a] += cvec<D>(i, a) > 0 ? g.v[j] : -g.v[j];
      Es[j] += real(cnorm2<D>(i)) * g.v[j];
    }
  });
  real E = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
#pragma unroll
    for (int a = 0; a < D; ++a) Jg[j][a] *= p.cj[j];
    E += p.cj2[j] * Es[j];
  }
  real rhot = 0, C = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    rhot += rho[j];
    C += rho[j] * p.invM[j];
  }
  // mixture velocity of f: total momentum is conserved by the collision, so
  // J(f) = J(g) + rho F / 2
  real u[D], u2 = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    real J = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) J += Jg[j][a];
    u[a] = (J + real(0.5) * rhot * p.F[a]) / rhot;
    u2 += u[a] * u[a];
  }
  const real T = (E - rhot * u2) / (real(D) * C);
  {
    // stability record: a non-finite or negative density or temperature
    // (NaN fails every comparison); all nodes that see it in one step store
    // the same step number, and a later step never overwrites it
    bool ok = T > real(0) && T < real(1e30) && u2 < real(1e30);
#pragma unroll
    for (int j = 0; j < NS; ++j) ok = ok && rho[j] >= real(0);
    if (!ok && b.status[0] == 0) {
      b.status[1] = b.status[2] + 1;
      b.status[0] = 1;
    }
  }
  // transport with floored mole fractions
  real Xh[NS], sX = 0, sMX = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    Xh[j] = fmax(rho[j] * p.invM[j] / C, real(1e-6));
    sX += Xh[j];
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    Xh[j] /= sX;
    sMX += p.M[j] * Xh[j];
  }
  const real lT = log(T / p.T_ref);
  const real CT = C * T;
  Rec<real, NR> fr;
  Rec<real, NX> fx;
  real tau2[NS];
  if (!p.lj) {
    // power laws: the viscosity ratios, hence Wilke's phi_jk, do not depend on T
    const real fmu = p.mu_T_exp == real(0) ? real(1) : exp(p.mu_T_exp * lT);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      real den = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) den += Xh[k] * p.wilke[j][k];
      const real tau1 = p.mu0[j] * fmu / (CT * den);  // Eq.(17)
      fr.v[fr_tau1(D, j)] = tau1;
      tau2[j] = tau1;
    }
  } else {
    // Eq.(26) with collision integrals: mu_j = mu0_j Omega_mu(T*_ref) sqrt(T/T_ref)
    // / Omega_mu(T*_j) (the reference factor is folded into mu0 on the host);
    // Wilke's phi_jk, Eq.(15) with the square, from these viscosities
    const real sq = sqrt(T / p.T_ref);
    real mu[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) mu[j] = p.mu0[j] * sq / lj_omega(p, b.lj_tab, T * p.lj_ie[j]);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      real den = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const real br = real(1) + sqrt(mu[j] / mu[k]) * sqrt(p.sqM[k] / p.sqM[j]);
        den += Xh[k] * br * br / sqrt(real(8) * (real(1) + p.M[j] * p.invM[k]));
      }
      const real tau1 = mu[j] / (CT * den);  // Eq.(17)
      fr.v[fr_tau1(D, j)] = tau1;
      tau2[j] = tau1;
    }
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) fr.v[fr_rho(D, j)] = rho[j];
  if (NS > 1) {
    // Eq.(27) with T^(3/2) and 1/p when collision integrals are on
    const real gD = p.lj ? sqrt(T / p.T_ref) * (T / p.T_ref) * (p.p_ref / CT)
                         : exp(p.D_T_exp * lT + p.D_p_exp * log(p.p_ref / CT));
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      real sum = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (k != j)
          sum += Xh[k] * p.invD0[j][k] *
                 (p.lj ? lj_omega(p, b.lj_tab + p.lj_n, T * sqrt(p.lj_ie[j] * p.lj_ie[k])) : real(1));
      const real Dj = gD * (real(1) - p.M[j] * Xh[j] / sMX) / sum;  // Eq.(8)
      tau2[j] = p.M[j] * Dj / T;                                    // Eq.(7)
    }
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) fx.v[fx_tau2(D, j)] = tau2[j];
#pragma unroll
  for (int a = 0; a < D; ++a) fr.v[fr_u(a)] = u[a];
  fr.v[fr_T(D)] = T;
  // Eq.(25) with Eq.(11): species momenta of f and U^c in closed form
  const bool cdiff = (p.flags & 1u) && NS > 1;
  real ediff = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    real num = 0, den = 0, K[NS], ah[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      ah[j] = real(0.5) / tau2[j];
      K[j] = (Jg[j][a] + ah[j] * rho[j] * u[a] + real(0.5) * rho[j] * p.F[a]) / (real(1) + ah[j]);
      num += ah[j] * (K[j] - rho[j] * u[a]);
      den += ah[j] * rho[j] / (real(1) + ah[j]);
    }
    const real Uc = cdiff ? num / den : real(0);
    fx.v[fx_Uc(a)] = Uc;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const real Jf = K[j] + ah[j] * rho[j] * Uc / (real(1) + ah[j]);
      const real uja = rho[j] > tiny<real>() ? Jf / rho[j] : u[a];
      fx.v[fx_uj(D, j, a)] = uja;
      ediff += rho[j] * (uja - u[a]) * (uja - u[a]);
    }
  }
  fx.v[fx_ediff(D)] = ediff;
  strec<real, NR>(b.FR, t, fr);
  strec<real, NX>(b.FX, t, fx);
}

template <bool FAST, typename real, typename PT, int D, int NS>
__device__ __forceinline__ void moments_block(const Params<real> &p, const Bufs<real, PT> &b, int cur,
                                              const WTab<real> &wtab, int lb) {
  const int first = FAST ? 0 : p.n_gas_fast, count = FAST ? p.n_gas_fast : p.n_gas - p.n_gas_fast;
  const int tl = lb * BLOCK + threadIdx.x;
  if (tl < count) moments_node<FAST, real, PT, D, NS>(p, b, cur, wtab, first + tl);
}
// one node list per launch (BF16 storage: there the combined kernel below
// ran 12 % slower on the 256^3 bed, the others gain from it)
template <bool FAST, typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK, 4) k_moments_list(Params<real> p, Bufs<real, PT> b, int cur) {
  __shared__ WTab<real> wtab;
  load_wtab_gas<real, NS>(p, wtab);
  const int count = FAST ? p.n_gas_fast : p.n_gas - p.n_gas_fast;
  const int nb = (count + BLOCK - 1) / BLOCK, lb = xcd_block(nb);
  if (lb >= nb) return;
  moments_block<FAST, real, PT, D, NS>(p, b, cur, wtab, lb);
}
// one launch over both node lists (the plain-stride blocks, then the
// periodic-wrap ones): the second list's blocks fill the first one's tail
template <typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK, 4) k_moments(Params<real> p, Bufs<real, PT> b, int cur) {
  __shared__ WTab<real> wtab;
  load_wtab_gas<real, NS>(p, wtab);
  const int nf = (p.n_gas_fast + BLOCK - 1) / BLOCK, nw = (p.n_gas - p.n_gas_fast + BLOCK - 1) / BLOCK;
  const int lb = xcd_block(nf + nw);
  if (lb >= nf + nw) return;
  if (lb < nf) moments_block<true, real, PT, D, NS>(p, b, cur, wtab, lb);
  else moments_block<false, real, PT, D, NS>(p, b, cur, wtab, lb - nf);
}

// ===========================================================================
// k_collide: streaming, sources, temperatures, equilibria and Eq.(24)
// ===========================================================================
// lattice-minus-Maxwellian third moment Q'_aaa of the equilibria
template <typename real>
__device__ inline real q_dev(real rho, real invM, real ua, real T) {
  return rho * invM * ua * (real(1) - real(3) * T) - rho * ua * ua * ua;
}
// lattice-minus-Maxwellian energy flux R'_ab of the equilibria
template <typename real, int D>
__device__ inline real r_dev(real rho, real invM, const real *u, real T, int a, int b) {
  if (a == b) {
    const real ua2 = u[a] * u[a];
    return rho * (T * (real(1) - real(3) * T) * invM * invM + ua2 * (real(1) - real(6) * T) * invM -
                  ua2 * ua2);
  }
  real u2 = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) u2 += u[c] * u[c];
  return rho * u[a] * u[b] * ((real(2) - real(D + 4) * T) * invM - u2);
}

// Equilibrium of Eq.(4)/(6) per unit density from the per-axis factors
// P0 = 1 - T - U^2, P+- = (T + U^2 +- U)/2 at the scaled velocity U =
// sqrt(M_j) u: a moving direction i (D2Q9 product; D3Q19 faces
// P_a (1 - 2T - U_b^2 - U_c^2), edges P_a P_b) ...
template <typename real, int D, int i>
__device__ inline real eq_moving(const real *U, real T) {
  if constexpr (D == 2) {
    constexpr int cx = cvec<D>(i, 0), cy = cvec<D>(i, 1);
    const real fx = cx == 0 ? real(1) - T - U[0] * U[0] : real(0.5) * (T + U[0] * U[0] + real(cx) * U[0]);
    const real fy = cy == 0 ? real(1) - T - U[1] * U[1] : real(0.5) * (T + U[1] * U[1] + real(cy) * U[1]);
    return fx * fy;
  } else if constexpr (is_face<D>(i)) {
    constexpr int a = edge_axis<D>(i, 0);
    constexpr int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    constexpr real sg = real(cvec<D>(i, a));
    return real(0.5) * (T + U[a] * U[a] + sg * U[a]) * (real(1) - real(2) * T - U[b1] * U[b1] - U[b2] * U[b2]);
  } else {
    constexpr int a0 = edge_axis<D>(i, 0), a1 = edge_axis<D>(i, 1);
    constexpr real s0 = real(cvec<D>(i, a0)), s1 = real(cvec<D>(i, a1));
    return real(0.25) * (T + U[a0] * U[a0] + s0 * U[a0]) * (T + U[a1] * U[a1] + s1 * U[a1]);
  }
}
// ... and the rest population (D3Q19: one minus all moving populations, in
// closed form)
template <typename real, int D>
__device__ inline real eq_rest(const real *U, real T) {
  if constexpr (D == 2) {
    return (real(1) - T - U[0] * U[0]) * (real(1) - T - U[1] * U[1]);
  } else {
    const real s0 = T + U[0] * U[0], s1 = T + U[1] * U[1], s2 = T + U[2] * U[2];
    const real q0 = U[0] * U[0], q1 = U[1] * U[1], q2 = U[2] * U[2];
    const real faces = s0 * (real(1) - real(2) * T - q1 - q2) + s1 * (real(1) - real(2) * T - q0 - q2) +
                       s2 * (real(1) - real(2) * T - q0 - q1);
    return real(1) - faces - (s0 * s1 + s0 * s2 + s1 * s2);
  }
}

// the collision's source node: the node itself (inlet and outlet nodes are
// set to equilibria instead)
struct SrcNode {
  int node, slot;
};

// Per-species constants of the collision at one node, for Eq.(24) in its
// difference form g+ = g - w (g - rho P*) - w (tau1/tau2) rho (P* - P^eq) +
// w tau1 S (P*, P^eq: equilibria per unit density; f* and f^eq differ only by
// the diffusion velocity, so their difference is formed directly), with the
// source moments pre-scaled by w tau1 and the species lattice speed.
template <typename real, int D>
struct SpeciesColl {
  real w, rho, a2;            // w = 2/(1 + 2 tau1), a2 = w (tau1/tau2) rho
  real Us[3];                 // sqrt(M_j) u_j (auxiliary-state velocity)
  real mS[D], PdS[D], YS[D];  // momentum, diagonal second moment, energy flux
  real PoS[3];                // off-diagonal second moments xy, xz, yz
  real eS;                    // energy (Prandtl term)
  real r_st, r_rest;          // rest population: rho P*_0 and a2 (P*_0 - P^eq_0) - w tau1 S_0
};

// Collision of all species at gas slot t (node sc.node, slot sc.slot == t).
template <typename real, typename PT, int D, int NS>
__device__ inline void collide_node(const Params<real> &p, const Bufs<real, PT> &b, int cur, const int t,
                                    const SrcNode sc) {
  constexpr int Q = lat_q<D>();
  constexpr int NR = fr_count(D, NS), NX = fx_count(D, NS);
  const int nsl = p.nsl;
  const int ss = sc.slot;
  // ---- the node's fields (pass 1) ----
  const Rec<real, NR> me = ldrec<real, NR>(b.FR, ss);
  const Rec<real, NX> mx = ldrec<real, NX>(b.FX, ss);
  real u[D];
#pragma unroll
  for (int a = 0; a < D; ++a) u[a] = me.v[fr_u(a)];
  const real Tt = me.v[fr_T(D)];
  real C = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) C += me.v[fr_rho(D, j)] * p.invM[j];
  // switches (uniform): 1 or 0
  const real kdiff = ((p.flags & 1u) && NS > 1) ? real(1) : real(0);
  const real kvisc = (p.flags & 2u) ? real(1) : real(0);
  const real kener = (p.flags & 4u) ? real(1) : real(0);
  const bool prc = (p.flags & 8u) != 0;  // Prandtl correction on
  // ---- source moments of every species ----
  real m[NS][D], Pd[NS][D], Po[NS][3], Y[NS][D], e[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const real rj = me.v[fr_rho(D, j)];
    const real tau2 = mx.v[fx_tau2(D, j)];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      m[j][a] = kdiff * rj * mx.v[fx_Uc(a)] / tau2 + rj * p.F[a];  // Eq.(12) + body force
      Pd[j][a] = real(2) * rj * u[a] * p.F[a];
      Y[j][a] = 0;
    }
    Po[j][0] = rj * (u[0] * p.F[1] + u[1] * p.F[0]);
    Po[j][1] = Po[j][2] = 0;
    if constexpr (D == 3) {
      Po[j][1] = rj * (u[0] * p.F[2] + u[2] * p.F[0]);
      Po[j][2] = rj * (u[1] * p.F[2] + u[2] * p.F[1]);
    }
    e[j] = 0;
  }
  const Addr<D> ad(sc.node, p);
  const int null_slot = p.n_gas + p.n_wall;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    // face neighbours along a: slot (the node itself when missing) and kind
    Rec<real, NR> nr[2];
    bool wall[2], miss[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int q = ad.face(p, a, s == 0 ? +1 : -1);
      const int ql = ld(b.slot_of, q >= 0 ? q : sc.node);  // unconditional load
      const int qs = q >= 0 ? ql : null_slot;
      wall[s] = qs >= p.n_gas && qs < null_slot;
      miss[s] = qs == null_slot || q == sc.node;
      nr[s] = ldrec<real, NR>(b.FR, miss[s] ? ss : qs);
    }
    real up[D], um[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      up[c] = nr[0].v[fr_u(c)];
      um[c] = nr[1].v[fr_u(c)];
    }
    const real Tp = nr[0].v[fr_T(D)], Tm = nr[1].v[fr_T(D)];
    const bool fp = !wall[0] && !miss[0], fm = !wall[1] && !miss[1];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const real iM = p.invM[j];
      const real rj = me.v[fr_rho(D, j)];
      const real rp = nr[0].v[fr_rho(D, j)], rm = nr[1].v[fr_rho(D, j)];
      // d_a Q'_aaa; a wall face carries no correction flux (mirror value)
      const real qx = q_dev<real>(rj, iM, u[a], Tt);
      const real qp = wall[0] ? -qx : q_dev<real>(rp, iM, up[a], Tp);
      const real qm = wall[1] ? -qx : q_dev<real>(rm, iM, um[a], Tm);
      Pd[j][a] += kvisc * real(0.5) * (qp - qm);
      if constexpr (D == 3) {
        // d_a of Q'_xyz = -rho u_x u_y u_z feeds the off-diagonal pair not containing a
        const real dq = real(0.5) * (-rp * up[0] * up[1] * up[2] + rm * um[0] * um[1] * um[2]);
        Po[j][2 - a] += kvisc * dq;  // a = x -> yz (2), y -> xz (1), z -> xy (0)
      }
      // energy-flux deviation R'_ca: the off-diagonal part as a source of
      // c_c c^2 moment d_a R'_ca; the diagonal (heat-conduction) part as
      // the energy source of the heat flux -tau1 d_a R'_aa in face-flux form
      // (face-averaged tau1, no flux through wall or missing faces)
#pragma unroll
      for (int c = 0; c < D; ++c)
        if (c != a)
          Y[j][c] += kener * real(0.5) * (r_dev<real, D>(rp, iM, up, Tp, c, a) - r_dev<real, D>(rm, iM, um, Tm, c, a));
      {
        const real Rx = r_dev<real, D>(rj, iM, u, Tt, a, a);
        const real t1x = me.v[fr_tau1(D, j)];
        const real gp = real(-0.5) * (t1x + nr[0].v[fr_tau1(D, j)]) * (r_dev<real, D>(rp, iM, up, Tp, a, a) - Rx);
        const real gm = real(-0.5) * (t1x + nr[1].v[fr_tau1(D, j)]) * (r_dev<real, D>(rm, iM, um, Tm, a, a) - Rx);
        e[j] += kener * ((fp ? gp : real(0)) + (fm ? gm : real(0)));
      }
      // Eq.(19)-(21), face-flux form; wall faces carry no correction flux
      const real kpr = prc ? p.kprj[j] : real(0);
      const real Kx = kpr * me.v[fr_tau1(D, j)] * rj * iM * Tt * iM;
      const real ep = real(0.5) * (Kx + kpr * nr[0].v[fr_tau1(D, j)] * rp * iM * Tp * iM) * (Tp - Tt);
      const real em = real(0.5) * (Kx + kpr * nr[1].v[fr_tau1(D, j)] * rm * iM * Tm * iM) * (Tm - Tt);
      e[j] += (fp ? ep : real(0)) + (fm ? em : real(0));
    }
  }
  // ---- temperatures of f (Eq.(25): T plus half the source energy) and of
  // the auxiliary state (quasi-equilibrium at fixed species momenta and energy)
  real esum = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    real trP = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) trP += Pd[j][a];
    esum += trP + e[j];
  }
  const real Tf = Tt + esum / (real(2 * D) * C);
  const real Tst = Tf - mx.v[fx_ediff(D)] / (real(D) * C);
  // ---- per-species constants ----
  SpeciesColl<real, D> sp[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    SpeciesColl<real, D> &c = sp[j];
    const real rj = me.v[fr_rho(D, j)];
    const real tau1 = me.v[fr_tau1(D, j)], tau2 = mx.v[fx_tau2(D, j)];
    const real w1 = real(2) / (real(1) + real(2) * tau1);
    const real r12 = tau1 / tau2;
    const real wt = w1 * tau1;
    c.w = w1;
    c.rho = rj;
    c.a2 = w1 * r12 * rj;
    const real ic = p.invcj[j], ic2 = ic * ic, ic3 = ic2 * ic;
    real trP = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      c.Us[a] = p.sqM[j] * mx.v[fx_uj(D, j, a)];
      c.mS[a] = wt * m[j][a] * ic;
      c.PdS[a] = wt * real(0.5) * Pd[j][a] * ic2;
      c.YS[a] = wt * Y[j][a] * ic3;
      trP += Pd[j][a];
    }
    if constexpr (D == 2) c.Us[2] = real(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) c.PoS[k] = wt * real(0.25) * Po[j][k] * ic2;
    c.eS = wt * e[j] * ic2 / real(2 * D);
    real Ue[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) Ue[a] = p.sqM[j] * u[a];
    const real ps0 = eq_rest<real, D>(c.Us, Tst), pe0 = eq_rest<real, D>(Ue, Tf);
    c.r_st = rj * ps0;
    c.r_rest = c.a2 * (ps0 - pe0) + wt * (trP + e[j]) * ic2;
  }
  // ---- streaming and collision, one direction at a time ----
  // (keep the scheduler from hoisting this phase's loads into the source
  // phase above, where most registers are already live)
  __builtin_amdgcn_sched_barrier(0);
  constexpr int RL = rec_len<PT>(NS);
  const PT *__restrict__ G = b.G[cur];
  PT *__restrict__ Gn = b.G[cur ^ 1];
  {
    const Rec<real, NS> g0 = pop_load<real, PT, D, NS>(p, G, ss, 0);  // rest: not streamed
    Rec<real, NS> o;
#pragma unroll
    for (int j = 0; j < NS; ++j) o.v[j] = g0.v[j] - sp[j].w * (g0.v[j] - sp[j].r_st) - sp[j].r_rest;
    pop_store_next<real, PT, D, NS>(p, Gn, t, 0, o);
  }
  static_for<1, Q>([&](auto ic_) __attribute__((always_inline)) {
    constexpr int i = decltype(ic_)::value;
    const Rec<real, NS> g = pop_load<real, PT, D, NS>(p, b.Gs + (size_t)i * nsl * RL, ss, i);
    Rec<real, NS> o;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const SpeciesColl<real, D> &c = sp[j];
      real Ue[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) Ue[a] = p.sqM[j] * u[a];
      const real pe = eq_moving<real, D, i>(Ue, Tf), ps = eq_moving<real, D, i>(c.Us, Tst);
      real S;
      if constexpr (is_face<D>(i)) {
        constexpr int a = edge_axis<D>(i, 0);
        constexpr real sg = real(cvec<D>(i, a));
        S = sg * c.mS[a] + c.PdS[a] - real(0.5) * sg * c.YS[a] + c.eS;
      } else {
        constexpr real kd = D == 2 ? real(0.25) : real(0.125);
        constexpr int a0 = edge_axis<D>(i, 0), a1 = edge_axis<D>(i, 1);
        constexpr int s0 = cvec<D>(i, a0), s1 = cvec<D>(i, a1);
        constexpr int po = D == 2 ? 0 : (a0 == 0 ? (a1 == 1 ? 0 : 1) : 2);
        S = -kd * (real(s0) * c.mS[a0] + real(s1) * c.mS[a1]) + real(s0 * s1) * c.PoS[po] +
            kd * (real(s0) * c.YS[a0] + real(s1) * c.YS[a1]);
      }
      o.v[j] = g.v[j] - c.w * (g.v[j] - c.rho * ps) - c.a2 * (ps - pe) + S;
    }
    pop_store_next<real, PT, D, NS>(p, Gn + (size_t)i * nsl * RL, t, i, o);
  });
}

// inlet node: equilibrium at the inlet state with the velocity of the first
// interior plane of its row (Sec. 6)
template <typename real, typename PT, int D, int NS>
__device__ inline void inlet_node(const Params<real> &p, const Bufs<real, PT> &b, int cur, int t,
                                  int node) {
  constexpr int Q = lat_q<D>();
  constexpr int NR = fr_count(D, NS);
  const int nsl = p.nsl;
  const int src = node - node % p.nx + 2;
  const bool ok = gaslike(b.kind[src]);
  const Rec<real, NR> fr = ldrec<real, NR>(b.FR, ok ? ld(b.slot_of, src) : t);
  constexpr int RL = rec_len<PT>(NS);
  PT *__restrict__ Gn = b.G[cur ^ 1];
  real U[NS][3];
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int a = 0; a < 3; ++a) U[j][a] = (ok && a < D) ? p.sqM[j] * fr.v[fr_u(a)] : real(0);
  {
    Rec<real, NS> o;
#pragma unroll
    for (int j = 0; j < NS; ++j) o.v[j] = p.rho_in[j] * eq_rest<real, D>(U[j], p.T_in);
    pop_store_next<real, PT, D, NS>(p, Gn, t, 0, o);
  }
  static_for<1, Q>([&](auto ic_) __attribute__((always_inline)) {
    constexpr int i = decltype(ic_)::value;
    Rec<real, NS> o;
#pragma unroll
    for (int j = 0; j < NS; ++j) o.v[j] = p.rho_in[j] * eq_moving<real, D, i>(U[j], p.T_in);
    pop_store_next<real, PT, D, NS>(p, Gn + (size_t)i * nsl * RL, t, i, o);
  });
}

// outlet node: equilibrium at the inlet pressure with the mole fractions,
// temperature and velocity of the last interior plane of its row (Sec. 6; a
// copy of the whole state would leave the outlet pressure free, and a
// body-force-driven flow would drain the domain)
template <typename real, typename PT, int D, int NS>
__device__ inline void outlet_node(const Params<real> &p, const Bufs<real, PT> &b, int cur, int t,
                                   int node) {
  constexpr int Q = lat_q<D>();
  constexpr int NR = fr_count(D, NS);
  constexpr int RL = rec_len<PT>(NS);
  const int nsl = p.nsl;
  const int src = node - node % p.nx + p.nx - 3;  // gas (checked with the geometry)
  const Rec<real, NR> fr = ldrec<real, NR>(b.FR, ld(b.slot_of, src));
  const real T = fr.v[fr_T(D)];
  real C = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) C += fr.v[fr_rho(D, j)] * p.invM[j];
  const real scale = p.p_in / (T * C);  // rho_j -> M_j X_j p_in / T
  PT *__restrict__ Gn = b.G[cur ^ 1];
  real U[NS][3], rj[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    rj[j] = fr.v[fr_rho(D, j)] * scale;
#pragma unroll
    for (int a = 0; a < 3; ++a) U[j][a] = a < D ? p.sqM[j] * fr.v[fr_u(a)] : real(0);
  }
  {
    Rec<real, NS> o;
#pragma unroll
    for (int j = 0; j < NS; ++j) o.v[j] = rj[j] * eq_rest<real, D>(U[j], T);
    pop_store_next<real, PT, D, NS>(p, Gn, t, 0, o);
  }
  static_for<1, Q>([&](auto ic_) __attribute__((always_inline)) {
    constexpr int i = decltype(ic_)::value;
    Rec<real, NS> o;
#pragma unroll
    for (int j = 0; j < NS; ++j) o.v[j] = rj[j] * eq_moving<real, D, i>(U[j], T);
    pop_store_next<real, PT, D, NS>(p, Gn + (size_t)i * nsl * RL, t, i, o);
  });
}

// one thread per gas node, all species, in slot order
// (FP32 arithmetic: at least 2 waves per SIMD, i.e. at most 256 VGPRs; the
// 16-bit storage variants would otherwise spill into AGPRs and run 1 wave)
template <typename real, typename PT, int D, int NS>
__device__ __forceinline__ void collide_block(const Params<real> &p, const Bufs<real, PT> &b, int cur, int lb) {
  const int t = lb * BLOCK + threadIdx.x;
  double work = 0.0;
  if (t < p.n_gas) {
    const int node = (int)b.gas_list[t];
    {
      // work of the body force on the gas at t this step, rho u.F (half the
      // trace of its source)
      constexpr int NR = fr_count(D, NS);
      const Rec<real, NR> at = ldrec<real, NR>(b.FR, t);
      real uf = 0, rt = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) uf += at.v[fr_u(a)] * p.F[a];
#pragma unroll
      for (int j = 0; j < NS; ++j) rt += at.v[fr_rho(D, j)];
      work = (double)(rt * uf);
    }
    const uint8_t k = b.kind[node];
    if (k == KIND_INLET) inlet_node<real, PT, D, NS>(p, b, cur, t, node);
    else if (k == KIND_OUTLET) outlet_node<real, PT, D, NS>(p, b, cur, t, node);
    else collide_node<real, PT, D, NS>(p, b, cur, t, SrcNode{node, t});
  }
  const double s = block_sum(work);
  if (threadIdx.x == 0 && s != 0.0) b.acc_work[lb] += s;
  // one step more completed (read by the next step's moments pass)
  if (lb == 0 && threadIdx.x == 0) b.status[2] += 1;
}
template <typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK, sizeof(real) == 4 ? 2 : 1) k_collide(Params<real> p, Bufs<real, PT> b, int cur) {
  // reversed: the streamed copy and moment records of the last blocks of
  // k_moments come first
  const int nb = (p.n_gas + BLOCK - 1) / BLOCK, lb = xcd_block_reversed(nb);
  if (lb >= nb) return;  // whole block: no barrier follows for it
  collide_block<real, PT, D, NS>(p, b, cur, lb);
}

// ===========================================================================
// k_solid: the heat step of the solid over an LDS tile with a one-node halo.
// MODE 0: forward Euler, Tout = Tin + a L Tin + source.  The Crank-Nicolson
// variant (the extension Sec. 5 recommends for a > 1/(2D)) solves
// T' - (a/2) L T' = T + (a/2) L T + source by Jacobi sweeps: MODE 1 writes
// that right-hand side, MODE 2 is one sweep Tin -> Tout, MODE 3 adds the
// new temperature's half of the Dirichlet-face heat.
// ===========================================================================
template <typename real, typename PT, int D, int MODE>
__device__ __forceinline__ void solid_pass(const Params<real> &p, const Bufs<real, PT> &b, const real *Tin,
                                           real *Tout, int tile) {
  constexpr int TX = SolidTile<D>::TX, TY = SolidTile<D>::TY, TZ = SolidTile<D>::TZ;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = D == 3 ? TZ + 2 : 1;
  __shared__ real sT[HZ * HY * HX];
  __shared__ uint8_t sK[HZ * HY * HX];  // 1 solid, 0 not solid, 2 outside a closed axis
  const int tilesX = (p.nx + TX - 1) / TX, tilesY = (p.ny + TY - 1) / TY;
  int bid = tile;
  const int bx = bid % tilesX;
  bid /= tilesX;
  const int by = bid % tilesY;
  const int bz = bid / tilesY;
  const int x0 = bx * TX - 1, y0 = by * TY - 1, z0 = D == 3 ? bz * TZ - 1 : 0;
  for (int q = threadIdx.x; q < HZ * HY * HX; q += BLOCK) {
    const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
    int x = x0 + hx, y = y0 + hy, z = z0 + hz;
    uint8_t k = 0;
    real v = 0;
    bool out = false;
    if (x < 0 || x >= p.nx) {
      if (p.per[0]) x = (x + p.nx) % p.nx;
      else out = true;
    }
    if (y < 0 || y >= p.ny) {
      if (p.per[1]) y = (y + p.ny) % p.ny;
      else out = true;
    }
    if (D == 3 && (z < 0 || z >= p.nz)) {
      if (p.per[2]) z = (z + p.nz) % p.nz;
      else out = true;
    }
    if (out) {
      k = 2;
    } else {
      const int nd = x + p.nx * (y + p.ny * z);
      const uint8_t kd = b.kind[nd];
      if (kd == KIND_SOLID || kd == KIND_WALL) {
        k = 1;
        v = Tin[nd];
      }
    }
    sK[q] = k;
    sT[q] = v;
  }
  __syncthreads();
  double bflux = 0.0;
  for (int q = threadIdx.x; q < TX * TY * TZ; q += BLOCK) {
    const int lx = q % TX, ly = (q / TX) % TY, lz = q / (TX * TY);
    const int x = x0 + 1 + lx, y = y0 + 1 + ly, z = z0 + (D == 3 ? 1 : 0) + lz;
    if (x >= p.nx || y >= p.ny || (D == 3 && z >= p.nz)) continue;
    const int hc = (lz + (D == 3 ? 1 : 0)) * HY * HX + (ly + 1) * HX + (lx + 1);
    if (sK[hc] != 1) continue;
    const real T = sT[hc];
    real lap = 0, bf = 0, nbs = 0, bcs = 0;
    int cnt = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int d = -1; d <= 1; d += 2) {
        const int off = a == 0 ? d : (a == 1 ? d * HX : d * HX * HY);
        const uint8_t kn = sK[hc + off];
        if (kn == 1) {
          lap += sT[hc + off] - T;
          nbs += sT[hc + off];
          ++cnt;
        } else if (kn == 2) {
          const int face = 2 * a + (d > 0 ? 1 : 0);
          if (p.has_bc[face]) {
            lap += p.T_bc[face] - T;
            bf += p.T_bc[face] - T;
            bcs += p.T_bc[face];
            ++cnt;
          }
        }
      }
    const int nd = x + p.nx * (y + p.ny * z);
    if constexpr (MODE == 0 || MODE == 1) {
      const real h = MODE == 0 ? p.alpha_s : real(0.5) * p.alpha_s;
      real Tn = T + h * lap;
      if (p.wall_mode == 0 && b.kind[nd] == KIND_WALL) {
        real qg;
        if (!p.eq48) {
          qg = -b.wall_dE[nd];  // flux-matched: the energy the wall gave the gas
        } else {
          // Eq.(48): kappa_f (T^f - T^s) per gas face neighbour, kappa_f =
          // sum_j (D+2) tau1_j C_j T / (2 M_j Pr_j) from the neighbour's
          // moments of this step (the solid then runs after them)
          qg = 0;
          const int NRr = fr_count(D, p.ns);
          const int c3[3] = {x, y, z}, lim[3] = {p.nx, p.ny, p.nz};
#pragma unroll
          for (int a = 0; a < D; ++a)
#pragma unroll
            for (int d = -1; d <= 1; d += 2) {
              const int off = a == 0 ? d : (a == 1 ? d * HX : d * HX * HY);
              if (sK[hc + off] != 0) continue;  // solid, or outside a closed axis
              int q[3] = {c3[0], c3[1], c3[2]};
              q[a] += d;
              q[a] = q[a] < 0 ? q[a] + lim[a] : (q[a] >= lim[a] ? q[a] - lim[a] : q[a]);
              const int ng = q[0] + p.nx * (q[1] + p.ny * q[2]);
              if (!gaslike(b.kind[ng])) continue;
              const real *fr = b.FR + (size_t)b.slot_of[ng] * NRr;
              const real Tf = fr[fr_T(D)];
              real kap = 0;
              for (int j = 0; j < p.ns; ++j)
                kap += p.kap[j] * fr[fr_tau1(D, j)] * fr[fr_rho(D, j)] * p.invM[j] * Tf * p.invM[j];
              qg += kap * (Tf - T);
            }
        }
        // the reaction heat: one reaction's -dH r, or several reactions' sum
        Tn += (p.n_rx == 1 ? -p.dH * b.wall_r[nd] + qg : b.wall_q[nd] + qg) * p.invCs;
      }
      if constexpr (MODE == 0) Tout[nd] = Tn;
      else b.cn_rhs[nd] = Tn;
      bflux += (double)(h * p.C_s * bf);
    } else if constexpr (MODE == 2) {
      const real h = real(0.5) * p.alpha_s;
      Tout[nd] = (b.cn_rhs[nd] + h * (nbs + bcs)) / (real(1) + h * real(cnt));
    } else {
      bflux += (double)(real(0.5) * p.alpha_s * p.C_s * bf);
    }
  }
  if constexpr (MODE != 2) {
    const double s = block_sum(bflux);
    if (threadIdx.x == 0 && s != 0.0) b.acc_bheat[tile] += s;
  }
}
template <typename real, typename PT, int D>
__device__ __forceinline__ void solid_block(const Params<real> &p, const Bufs<real, PT> &b, int cur, int tile) {
  solid_pass<real, PT, D, 0>(p, b, b.Ts[cur], b.Ts[cur ^ 1], tile);
}
template <typename real, typename PT, int D, int MODE>
__global__ void __launch_bounds__(BLOCK) k_solid_pass(Params<real> p, Bufs<real, PT> b, const real *Tin,
                                                      real *Tout) {
  solid_pass<real, PT, D, MODE>(p, b, Tin, Tout, blockIdx.x);
}
template <typename real, typename PT, int D>
__global__ void __launch_bounds__(BLOCK) k_solid(Params<real> p, Bufs<real, PT> b, int cur) {
  solid_block<real, PT, D>(p, b, cur, blockIdx.x);
}


// ===========================================================================
// k_observe: FP64 partial sums per block.  Slots per block: [0, NS) species
// mass; then e_gas, e_solid, T_min, T_max, u_max, rho_min, Ts_min, Ts_max,
// bad.  Gas and wall populations are read per slot, the solid per node.
// ===========================================================================
template <typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK) k_observe(Params<real> p, Bufs<real, PT> b, int cur) {
  constexpr int Q = lat_q<D>();
  constexpr int NP = NS + 9;
  constexpr int S_EG = NS, S_ES = NS + 1, S_TMIN = NS + 2, S_TMAX = NS + 3, S_UMAX = NS + 4,
                S_RMIN = NS + 5, S_TSMIN = NS + 6, S_TSMAX = NS + 7, S_BAD = NS + 8;
  __shared__ double sh[NP][BLOCK];
  double acc[NP];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  acc[S_EG] = acc[S_ES] = acc[S_UMAX] = acc[S_BAD] = 0.0;
  acc[S_TMIN] = acc[S_RMIN] = acc[S_TSMIN] = 1e300;
  acc[S_TMAX] = acc[S_TSMAX] = -1e300;
  constexpr int RL = rec_len<PT>(NS);
  const PT *G = b.G[cur];
  const int n = p.n, nsl = p.nsl;
  const int gid = blockIdx.x * BLOCK + threadIdx.x, stride = gridDim.x * BLOCK;
  for (int node = gid; node < n; node += stride) {
    const uint8_t k = b.kind[node];
    if (k == KIND_SOLID || k == KIND_WALL) {
      const double ts = (double)b.Ts[cur][node];
      acc[S_ES] += (double)p.C_s * ts;
      acc[S_TSMIN] = fmin(acc[S_TSMIN], ts);
      acc[S_TSMAX] = fmax(acc[S_TSMAX], ts);
      if (!(ts > 0.0) || !isfinite(ts)) acc[S_BAD] = 1.0;
    }
  }
  for (int s = gid; s < p.n_gas + p.n_wall; s += stride) {
    const bool gas = s < p.n_gas;
    const uint32_t em = gas ? ~0u : b.wem[s - p.n_gas];
    double rj[NS], Ej[NS], Jj[NS][3];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      rj[j] = Ej[j] = 0.0;
      Jj[j][0] = Jj[j][1] = Jj[j][2] = 0.0;
    }
    for (int i = 0; i < Q; ++i) {
      if (!(em & (1u << i))) continue;
      const Rec<real, NS> rec = pop_load<real, PT, D, NS>(p, G + (size_t)i * nsl * RL, s, i);
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const double gv = (double)rec.v[j];
        if (!isfinite(gv)) acc[S_BAD] = 1.0;
        rj[j] += gv;
        Ej[j] += (double)cnorm2<D>(i) * gv;
#pragma unroll
        for (int a = 0; a < 3; ++a) Jj[j][a] += (double)cvec<D>(i, a) * gv;
      }
    }
    double E = 0, rhot = 0, C = 0, J[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      acc[j] += rj[j];
      E += (double)p.cj2[j] * Ej[j];
#pragma unroll
      for (int a = 0; a < 3; ++a) J[a] += (double)p.cj[j] * Jj[j][a];
      if (gas) {
        rhot += rj[j];
        C += rj[j] / (double)p.M[j];
        acc[S_RMIN] = fmin(acc[S_RMIN], rj[j]);
      }
    }
    acc[S_EG] += 0.5 * E;
    if (gas) {
      const double u2 = (J[0] * J[0] + J[1] * J[1] + J[2] * J[2]) / (rhot * rhot);
      const double T = (E - rhot * u2) / (D * C);
      acc[S_TMIN] = fmin(acc[S_TMIN], T);
      acc[S_TMAX] = fmax(acc[S_TMAX], T);
      acc[S_UMAX] = fmax(acc[S_UMAX], sqrt(u2));
      if (!(T > 0.0) || !(rhot > 0.0)) acc[S_BAD] = 1.0;
    }
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const int o = threadIdx.x + s;
#pragma unroll
      for (int k = 0; k < NS + 2; ++k) sh[k][threadIdx.x] += sh[k][o];
      sh[S_TMIN][threadIdx.x] = fmin(sh[S_TMIN][threadIdx.x], sh[S_TMIN][o]);
      sh[S_TMAX][threadIdx.x] = fmax(sh[S_TMAX][threadIdx.x], sh[S_TMAX][o]);
      sh[S_UMAX][threadIdx.x] = fmax(sh[S_UMAX][threadIdx.x], sh[S_UMAX][o]);
      sh[S_RMIN][threadIdx.x] = fmin(sh[S_RMIN][threadIdx.x], sh[S_RMIN][o]);
      sh[S_TSMIN][threadIdx.x] = fmin(sh[S_TSMIN][threadIdx.x], sh[S_TSMIN][o]);
      sh[S_TSMAX][threadIdx.x] = fmax(sh[S_TSMAX][threadIdx.x], sh[S_TSMAX][o]);
      sh[S_BAD][threadIdx.x] = fmax(sh[S_BAD][threadIdx.x], sh[S_BAD][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NP; ++k) b.partials[(size_t)blockIdx.x * NP + k] = sh[k][0];
}

// ===========================================================================
// k_residual: change of the fields since the last snapshot, for the steady-
// state test.  FP64 partial sums per block over the gas slots (mole fractions
// X_j, temperature, velocity) and the solid nodes (T^s): sum (q - q_snap)^2
// and sum q^2 per group, 8 values per block; then the snapshot is replaced.
// ===========================================================================
template <typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK) k_residual(Params<real> p, Bufs<real, PT> b, int cur) {
  constexpr int NR = fr_count(D, NS), NSN = sn_count(D, NS);
  __shared__ double sh[8][BLOCK];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int gid = blockIdx.x * BLOCK + threadIdx.x, stride = gridDim.x * BLOCK;
  for (int t = gid; t < p.n_gas; t += stride) {
    const Rec<real, NR> fr = ldrec<real, NR>(b.FR, t);
    Rec<real, NSN> q;
    real C = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) C += fr.v[fr_rho(D, j)] * p.invM[j];
#pragma unroll
    for (int j = 0; j < NS; ++j) q.v[j] = fr.v[fr_rho(D, j)] * p.invM[j] / C;
    q.v[NS] = fr.v[fr_T(D)];
#pragma unroll
    for (int a = 0; a < D; ++a) q.v[NS + 1 + a] = fr.v[fr_u(a)];
    const Rec<real, NSN> o = ldrec<real, NSN>(b.snap, t);
#pragma unroll
    for (int k = 0; k < NSN; ++k) {
      const int g = k < NS ? 0 : (k == NS ? 1 : 2);
      const double d = (double)q.v[k] - (double)o.v[k];
      acc[2 * g] += d * d;
      acc[2 * g + 1] += (double)q.v[k] * (double)q.v[k];
    }
    strec<real, NSN>(b.snap, t, q);
  }
  for (int node = gid; node < p.n; node += stride) {
    const uint8_t k = b.kind[node];
    if (!(k == KIND_SOLID || k == KIND_WALL)) continue;
    const real ts = b.Ts[cur][node];
    const double d = (double)ts - (double)b.snap_ts[node];
    acc[6] += d * d;
    acc[7] += (double)ts * (double)ts;
    b.snap_ts[node] = ts;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < 8; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) b.partials[(size_t)blockIdx.x * 8 + k] = sh[k][0];
}

// ===========================================================================
// batched persistent kernels: many independent domains (samples) advance in
// one launch per kernel.  Each sample has its own Params and Bufs in device
// memory; a work list holds (sample, logical block) pairs for every launch
// kind.  The work list is split into 8 contiguous runs, one per XCD, and the
// workgroups of an XCD walk their run in order, so neighbouring blocks of
// one sample share that XCD's L2 as in the single-domain launches.
// ===========================================================================
template <typename F>
__device__ __forceinline__ void for_items(const int2 *__restrict__ items, int n, F &&f) {
  const int per = (n + NXCD - 1) / NXCD;
  // gridDim.x is a multiple of NXCD: a workgroup keeps its XCD (q % NXCD)
  for (int q = (int)blockIdx.x; q < per * NXCD; q += (int)gridDim.x) {
    const int L = (q % NXCD) * per + q / NXCD;
    if (L < n) f(items[L]);
  }
}

template <bool FAST, bool HALF, bool MULTI, typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK) kb_wall(const Params<real> *__restrict__ P,
                                                 const Bufs<real, PT> *__restrict__ B,
                                                 const int2 *__restrict__ items, const int *__restrict__ count,
                                                 int cur) {
  __shared__ WTab<real> wtab;
  int prev = -1;
  for_items(items, *count, [&](int2 it) {
    if (it.x != prev) {
      __syncthreads();  // every thread is done with the previous sample's table
      load_wtab<real, NS>(P[it.x], wtab);
      prev = it.x;
    }
    wall_block<FAST, HALF, MULTI, real, PT, D, NS>(P[it.x], B[it.x], cur, wtab, it.y);
  });
}

template <bool FAST, typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK, 4) kb_moments(const Params<real> *__restrict__ P,
                                                    const Bufs<real, PT> *__restrict__ B,
                                                    const int2 *__restrict__ items,
                                                    const int *__restrict__ count, int cur) {
  __shared__ WTab<real> wtab;
  int prev = -1;
  for_items(items, *count, [&](int2 it) {
    if (it.x != prev) {
      __syncthreads();
      load_wtab_gas<real, NS>(P[it.x], wtab);
      prev = it.x;
    }
    moments_block<FAST, real, PT, D, NS>(P[it.x], B[it.x], cur, wtab, it.y);
  });
}

template <typename real, typename PT, int D, int NS>
__global__ void __launch_bounds__(BLOCK, sizeof(real) == 4 ? 2 : 1)
    kb_collide(const Params<real> *__restrict__ P, const Bufs<real, PT> *__restrict__ B,
               const int2 *__restrict__ items, const int *__restrict__ count, int cur) {
  for_items(items, *count, [&](int2 it) { collide_block<real, PT, D, NS>(P[it.x], B[it.x], cur, it.y); });
}

template <typename real, typename PT, int D>
__global__ void __launch_bounds__(BLOCK) kb_solid(const Params<real> *__restrict__ P,
                                                  const Bufs<real, PT> *__restrict__ B,
                                                  const int2 *__restrict__ items, const int *__restrict__ count,
                                                  int cur) {
  for_items(items, *count, [&](int2 it) {
    __syncthreads();  // the LDS tile of the previous item has been consumed
    solid_block<real, PT, D>(P[it.x], B[it.x], cur, it.y);
  });
}

// Crank-Nicolson solid of a batch: MODE 1 the right-hand side, MODE 2 Jacobi
// sweep `it` of `max_it` (a sample with k = cn_iters sweeps takes the last k,
// from T^s into the buffers the single-domain step uses, so that its last
// sweep lands in Ts[cur ^ 1]), MODE 3 the new temperature's face heat.
template <typename real, typename PT, int D, int MODE>
__global__ void __launch_bounds__(BLOCK) kb_solid_cn(const Params<real> *__restrict__ P,
                                                     const Bufs<real, PT> *__restrict__ B,
                                                     const int2 *__restrict__ items, const int *__restrict__ count,
                                                     int cur, int it, int max_it) {
  for_items(items, *count, [&](int2 item) {
    __syncthreads();  // the LDS tile of the previous item has been consumed
    const Params<real> &p = P[item.x];
    const Bufs<real, PT> &b = B[item.x];
    if constexpr (MODE == 1) {
      solid_pass<real, PT, D, 1>(p, b, b.Ts[cur], b.cn_tmp, item.y);
    } else if constexpr (MODE == 2) {
      const int li = it - (max_it - p.cn_iters);  // uniform over the workgroup
      if (li >= 0) {
        auto buf = [&](int l) { return ((p.cn_iters - 1 - l) % 2 == 0) ? b.Ts[cur ^ 1] : b.cn_tmp; };
        solid_pass<real, PT, D, 2>(p, b, li == 0 ? b.Ts[cur] : buf(li - 1), buf(li), item.y);
      }
    } else {
      solid_pass<real, PT, D, 3>(p, b, b.Ts[cur ^ 1], b.cn_tmp, item.y);
    }
  });
}

// ===========================================================================
// launchers
// ===========================================================================
// One time step.  Dependencies within the step: the collision needs the
// moments (same step) and the wall's state records (same step); the solid
// needs the wall's rate and energy exchange.  The wall reads the previous
// step's gas populations and writes the wall slots of the other buffer, which
// only the next step's moments read, so the wall (then the solid) can run on
// a second stream beside the moments (then the collision).
template <typename real, typename PT, int D, int NS>
inline hipError_t step_impl(const Params<real> &p, const Bufs<real, PT> &b, int cur,
                            LaunchInfo &li) {
  const int gwf = (p.n_wall_fast + BLOCK - 1) / BLOCK, gws = (p.n_wall - p.n_wall_fast + BLOCK - 1) / BLOCK;
  const int ggf = (p.n_gas_fast + BLOCK - 1) / BLOCK, ggs = (p.n_gas - p.n_gas_fast + BLOCK - 1) / BLOCK;
  hipStream_t st = li.stream;
  const bool two = li.side != nullptr;
  hipStream_t sw = two ? li.side : st;  // stream of the wall and solid kernels
  auto mark = [&](int k, int which, hipStream_t s) {
    if (li.events) {
      (void)hipEventRecord(li.events[2 * k + which], s);
      li.recorded[k] = true;
    }
  };
  const dim3 blk(BLOCK);
  if (two) {
    // everything enqueued before on the main stream (the previous step's
    // collision among it) precedes this step's wall kernel
    (void)hipEventRecord(li.ev_fork, st);
    (void)hipStreamWaitEvent(sw, li.ev_fork, 0);
  }
  mark(K_WALL_ID, 0, sw);
  // the wall variants: half-way wall and several reactions, as compile-time flags
  auto wall = [&](auto half, auto multi) {
    constexpr bool H = decltype(half)::value, MU = decltype(multi)::value;
    if (gwf > 0) hipLaunchKernelGGL((k_wall<true, H, MU, real, PT, D, NS>), dim3(xcd_grid(gwf)), blk, 0, sw, p, b, cur);
    if (gws > 0) hipLaunchKernelGGL((k_wall<false, H, MU, real, PT, D, NS>), dim3(xcd_grid(gws)), blk, 0, sw, p, b, cur);
  };
  const bool multi = p.n_rx > 1;
  if (!p.halfway && !multi) wall(std::false_type{}, std::false_type{});
  else if (p.halfway && !multi) wall(std::true_type{}, std::false_type{});
  else if (!p.halfway) wall(std::false_type{}, std::true_type{});
  else wall(std::true_type{}, std::true_type{});
  mark(K_WALL_ID, 1, sw);
  if (two) (void)hipEventRecord(li.ev_wall, sw);
  // the solid step: forward Euler, or Crank-Nicolson by p.cn_iters Jacobi
  // sweeps from T (right-hand side first, the last sweep into Ts[cur ^ 1])
  auto solid = [&](hipStream_t s) {
    const int tiles = solid_tiles<D>(p.nx, p.ny, p.nz);
    mark(K_SOLID_ID, 0, s);
    if (!p.solid_cn) {
      hipLaunchKernelGGL((k_solid<real, PT, D>), dim3(tiles), blk, 0, s, p, b, cur);
    } else {
      hipLaunchKernelGGL((k_solid_pass<real, PT, D, 1>), dim3(tiles), blk, 0, s, p, b, b.Ts[cur], b.cn_tmp);
      const real *src = b.Ts[cur];
      for (int it = 0; it < p.cn_iters; ++it) {
        real *dst = ((p.cn_iters - 1 - it) % 2 == 0) ? b.Ts[cur ^ 1] : b.cn_tmp;
        hipLaunchKernelGGL((k_solid_pass<real, PT, D, 2>), dim3(tiles), blk, 0, s, p, b, src, dst);
        src = dst;
      }
      hipLaunchKernelGGL((k_solid_pass<real, PT, D, 3>), dim3(tiles), blk, 0, s, p, b, b.Ts[cur ^ 1], b.cn_tmp);
    }
    mark(K_SOLID_ID, 1, s);
  };
  // the Eq.(48) coupling reads the gas moments of this step: its solid step
  // runs after them, on the main stream
  if (two && li.n_solid > 0 && !p.eq48) solid(sw);
  // the half-way wall reads the gas nodes' moment records of the previous
  // step, which the moments kernel overwrites
  if (two && p.halfway) (void)hipStreamWaitEvent(st, li.ev_wall, 0);
  mark(K_MOMENTS_ID, 0, st);
  if constexpr (std::is_same_v<PT, __bf16>) {
    if (ggf > 0)
      hipLaunchKernelGGL((k_moments_list<true, real, PT, D, NS>), dim3(xcd_grid(ggf)), blk, 0, st, p, b, cur);
    if (ggs > 0)
      hipLaunchKernelGGL((k_moments_list<false, real, PT, D, NS>), dim3(xcd_grid(ggs)), blk, 0, st, p, b, cur);
  } else if (ggf + ggs > 0) {
    hipLaunchKernelGGL((k_moments<real, PT, D, NS>), dim3(xcd_grid(ggf + ggs)), blk, 0, st, p, b, cur);
  }
  mark(K_MOMENTS_ID, 1, st);
  if (two) (void)hipStreamWaitEvent(st, li.ev_wall, 0);
  mark(K_COLLIDE_ID, 0, st);
  const int gg = (p.n_gas + BLOCK - 1) / BLOCK;
  if (gg > 0) hipLaunchKernelGGL((k_collide<real, PT, D, NS>), dim3(xcd_grid(gg)), blk, 0, st, p, b, cur);
  mark(K_COLLIDE_ID, 1, st);
  if (two) {
    // join: the step is complete on the main stream
    (void)hipEventRecord(li.ev_solid, sw);
    (void)hipStreamWaitEvent(st, li.ev_solid, 0);
  }
  if ((!two || p.eq48) && li.n_solid > 0) solid(st);
  return hipGetLastError();
}

// A batched step: the launch kinds in step order; with a side stream the
// wall and solid kinds run there beside the moments and collision kinds (the
// same dependencies as the single-domain step).
template <typename real, typename PT, int D, int NS>
inline hipError_t batch_step_impl(const BatchLaunch &bl, int cur) {
  const dim3 blk(BLOCK);
  const auto *P = static_cast<const Params<real> *>(bl.params);
  const auto *B = static_cast<const Bufs<real, PT> *>(bl.bufs);
  hipStream_t st = bl.stream;
  const bool two = bl.side != nullptr;
  hipStream_t sw = two ? bl.side : st;
  auto go = [&](int k) { return bl.grid[k] > 0 && bl.max_items[k] > 0; };
  if (two) {
    (void)hipEventRecord(bl.ev_fork, st);
    (void)hipStreamWaitEvent(sw, bl.ev_fork, 0);
  }
  // the solid step: forward Euler, or Crank-Nicolson (right-hand side, the
  // largest sample's number of Jacobi sweeps, face heat)
  auto solid = [&](hipStream_t s) {
    const dim3 g(bl.grid[BL_SOLID]);
    const int2 *items = bl.items[BL_SOLID];
    const int *cnt = bl.count + BL_SOLID;
    if (bl.cn_iters == 0) {
      hipLaunchKernelGGL((kb_solid<real, PT, D>), g, blk, 0, s, P, B, items, cnt, cur);
      return;
    }
    hipLaunchKernelGGL((kb_solid_cn<real, PT, D, 1>), g, blk, 0, s, P, B, items, cnt, cur, 0, bl.cn_iters);
    for (int it = 0; it < bl.cn_iters; ++it)
      hipLaunchKernelGGL((kb_solid_cn<real, PT, D, 2>), g, blk, 0, s, P, B, items, cnt, cur, it, bl.cn_iters);
    hipLaunchKernelGGL((kb_solid_cn<real, PT, D, 3>), g, blk, 0, s, P, B, items, cnt, cur, 0, bl.cn_iters);
  };
  // the wall variants (half-way wall, several reactions) as compile-time flags
  auto wall = [&](auto half, auto multi) {
    constexpr bool H = decltype(half)::value, MU = decltype(multi)::value;
    if (go(BL_WALL_FAST))
      hipLaunchKernelGGL((kb_wall<true, H, MU, real, PT, D, NS>), dim3(bl.grid[BL_WALL_FAST]), blk, 0, sw, P, B,
                         bl.items[BL_WALL_FAST], bl.count + BL_WALL_FAST, cur);
    if (go(BL_WALL_SLOW))
      hipLaunchKernelGGL((kb_wall<false, H, MU, real, PT, D, NS>), dim3(bl.grid[BL_WALL_SLOW]), blk, 0, sw, P, B,
                         bl.items[BL_WALL_SLOW], bl.count + BL_WALL_SLOW, cur);
  };
  if (!bl.halfway && !bl.multi) wall(std::false_type{}, std::false_type{});
  else if (bl.halfway && !bl.multi) wall(std::true_type{}, std::false_type{});
  else if (!bl.halfway) wall(std::false_type{}, std::true_type{});
  else wall(std::true_type{}, std::true_type{});
  if (two) {
    (void)hipEventRecord(bl.ev_wall, sw);
    // the Eq.(48) coupling reads this step's gas moments: its solid step runs
    // after them, on the main stream
    if (go(BL_SOLID) && !bl.eq48) solid(sw);
    (void)hipEventRecord(bl.ev_solid, sw);
    // the half-way wall reads the moment records the moments kernel overwrites
    if (bl.halfway) (void)hipStreamWaitEvent(st, bl.ev_wall, 0);
  }
  if (go(BL_GAS_FAST))
    hipLaunchKernelGGL((kb_moments<true, real, PT, D, NS>), dim3(bl.grid[BL_GAS_FAST]), blk, 0, st, P, B,
                       bl.items[BL_GAS_FAST], bl.count + BL_GAS_FAST, cur);
  if (go(BL_GAS_SLOW))
    hipLaunchKernelGGL((kb_moments<false, real, PT, D, NS>), dim3(bl.grid[BL_GAS_SLOW]), blk, 0, st, P, B,
                       bl.items[BL_GAS_SLOW], bl.count + BL_GAS_SLOW, cur);
  if (two) (void)hipStreamWaitEvent(st, bl.ev_wall, 0);
  if (go(BL_COLLIDE))
    hipLaunchKernelGGL((kb_collide<real, PT, D, NS>), dim3(bl.grid[BL_COLLIDE]), blk, 0, st, P, B,
                       bl.items[BL_COLLIDE], bl.count + BL_COLLIDE, cur);
  if (two) {
    (void)hipStreamWaitEvent(st, bl.ev_solid, 0);
    if (go(BL_SOLID) && bl.eq48) solid(st);
  } else if (go(BL_SOLID)) {
    solid(st);
  }
  return hipGetLastError();
}

template <typename real, typename PT, int D, int NS>
inline hipError_t residual_impl(const Params<real> &p, const Bufs<real, PT> &b, int cur, int blocks,
                                hipStream_t st) {
  hipLaunchKernelGGL((k_residual<real, PT, D, NS>), dim3(blocks), dim3(BLOCK), 0, st, p, b, cur);
  return hipGetLastError();
}

template <typename real, typename PT, int D, int NS>
inline hipError_t observe_impl(const Params<real> &p, const Bufs<real, PT> &b, int cur, int blocks,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_observe<real, PT, D, NS>), dim3(blocks), dim3(BLOCK), 0, st, p, b, cur);
  return hipGetLastError();
}

// species-count dispatch for one (precision, lattice); FDLBM_NS_CASES lists
// the species counts this translation unit instantiates
template <typename real, typename PT, int D>
hipError_t batch_step_lat(int ns, const BatchLaunch &bl, int cur) {
  switch (ns) {
#define FDLBM_CASE(k) \
  case k:             \
    return batch_step_impl<real, PT, D, k>(bl, cur);
    FDLBM_NS_CASES
#undef FDLBM_CASE
  }
  return hipErrorInvalidValue;
}

template <typename real, typename PT, int D>
hipError_t step_lat(const Params<real> &p, const Bufs<real, PT> &b, int cur, LaunchInfo &li) {
  switch (p.ns) {
#define FDLBM_CASE(k) \
  case k:             \
    return step_impl<real, PT, D, k>(p, b, cur, li);
    FDLBM_NS_CASES
#undef FDLBM_CASE
  }
  return hipErrorInvalidValue;
}

template <typename real, typename PT, int D>
hipError_t residual_lat(const Params<real> &p, const Bufs<real, PT> &b, int cur, int blocks,
                        hipStream_t st) {
  switch (p.ns) {
#define FDLBM_CASE(k) \
  case k:             \
    return residual_impl<real, PT, D, k>(p, b, cur, blocks, st);
    FDLBM_NS_CASES
#undef FDLBM_CASE
  }
  return hipErrorInvalidValue;
}

template <typename real, typename PT, int D>
hipError_t observe_lat(const Params<real> &p, const Bufs<real, PT> &b, int cur, int blocks,
                       hipStream_t st) {
  switch (p.ns) {
#define FDLBM_CASE(k) \
  case k:             \
    return observe_impl<real, PT, D, k>(p, b, cur, blocks, st);
    FDLBM_NS_CASES
#undef FDLBM_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace fdlbm
