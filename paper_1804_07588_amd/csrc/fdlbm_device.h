// Device-side definitions shared by the kernels and the host library:
// lattice tables, the parameter block passed to every kernel, the workspace
// pointer block, and the closed forms of the equilibria (Eq.(4), Eq.(6)) and
// of the correction-source shapes (Eq.(13) and the deviation corrections).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdlbm {

constexpr int MAXS = 8;     // species slots in the parameter block
constexpr int MAXR = 4;     // surface reactions per wall node
// reaction table (several reactions): per reaction k0, E_a / (R T_ref),
// T_ref, dH, then the stoichiometry nu_j and the orders of MAXS species
constexpr int RX_K0 = 0, RX_EA = 1, RX_TREF = 2, RX_DH = 3, RX_NU = 4, RX_ORD = 4 + MAXS, RXS = 4 + 2 * MAXS;
constexpr int MAX_NS = 6;   // species counts the kernels are instantiated for
constexpr int BLOCK = 256;  // threads per block of the list kernels

// ---------------------------------------------------------------------------
// lattice tables.  D2Q9 in the order of Eq.(2); D3Q19: rest, +x, -x, +y, -y,
// +z, -z, then the xy, xz, yz edges, each (+,+), (-,+), (-,-), (+,-).
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ constexpr int lat_q() {
  return D == 2 ? 9 : 19;
}

template <int D>
__host__ __device__ constexpr int cvec(int i, int a) {
  constexpr int c2[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                            {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  constexpr int c3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                             {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, 1, 0}, {-1, -1, 0},
                             {1, -1, 0}, {1, 0, 1},  {-1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                             {0, 1, 1},  {0, -1, 1}, {0, -1, -1}, {0, 1, -1}};
  return D == 2 ? c2[i][a] : c3[i][a];
}

template <int D>
__host__ __device__ constexpr int cnorm2(int i) {
  return cvec<D>(i, 0) * cvec<D>(i, 0) + cvec<D>(i, 1) * cvec<D>(i, 1) +
         cvec<D>(i, 2) * cvec<D>(i, 2);
}

// streaming stencil classes (3 bits per moving direction in the class word):
// 0 central (taps x-2e, x-e, x), 1 forward (x-e, x, x+e), 2 backward
// (x-e, x-2e, x-3e), 3 two-point (x-e, x), 4 two-point (x-2e, x-e),
// 5 one-point (x-e), 6 one-point (x), 7 not a destination.
constexpr int CLS_NONE = 7;
__host__ __device__ constexpr int stencil_ntaps(int cls) {
  return cls <= 2 ? 3 : (cls <= 4 ? 2 : 1);
}
__host__ __device__ constexpr int stencil_off(int cls, int k) {
  constexpr int off[7][3] = {{-2, -1, 0}, {-1, 0, 1}, {-1, -2, -3}, {-1, 0, 0},
                             {-2, -1, 0}, {-1, 0, 0}, {0, 0, 0}};
  return off[cls][k];
}

// tile of the solid heat kernel (one block, one-node halo in LDS)
template <int D>
struct SolidTile;
template <>
struct SolidTile<2> {
  static constexpr int TX = 32, TY = 8, TZ = 1;
};
template <>
struct SolidTile<3> {
  static constexpr int TX = 16, TY = 4, TZ = 4;
};
template <int D>
__host__ __device__ inline int solid_tiles(int nx, int ny, int nz) {
  return ((nx + SolidTile<D>::TX - 1) / SolidTile<D>::TX) * ((ny + SolidTile<D>::TY - 1) / SolidTile<D>::TY) *
         ((nz + SolidTile<D>::TZ - 1) / SolidTile<D>::TZ);
}

// ---------------------------------------------------------------------------
// parameter block (by value to every kernel)
// ---------------------------------------------------------------------------
template <typename real>
struct Params {
  int ns, nx, ny, nz, n;
  int per[3];
  int inout;
  unsigned flags;
  int wall_mode;
  int n_gas, n_wall;
  int nsl;                          // slot stride of the per-slot arrays (>= n_gas + n_wall + 1)
  int n_gas_fast, n_wall_fast;      // leading list entries whose taps never wrap
  int slot_off_gas, slot_off_wall;  // accumulator block offsets of the wrapping launches
  // species
  real M[MAXS], invM[MAXS], sqM[MAXS], cj[MAXS], cj2[MAXS], invcj[MAXS];
  real wint[MAXS][7][3];           // stencil weights per species and class
  real mu0[MAXS], mu_T_exp;
  real wilke[MAXS][MAXS];          // phi_jk of Eq.(15) (temperature independent)
  real invD0[MAXS][MAXS];          // 1 / Djk0
  real D_T_exp, D_p_exp, T_ref, p_ref;
  real kprj[MAXS];                 // (D+2)(1/Pr_j - 1) per species
  // Lennard-Jones transport: on, table length, grid origin and 1/spacing of
  // T*, T_unit / eps_j per species
  int lj, lj_n;
  real lj_t0, lj_idt;
  real lj_ie[MAXS];
  // solid
  real alpha_s, invCs, C_s;
  int solid_cn, cn_iters;          // Crank-Nicolson solid: on, Jacobi sweeps per step
  real T_bc[6];
  int has_bc[6];
  // reaction
  real nu[MAXS], k0, ea, T_ref_rxn, dH, T_iso, tol;
  int order[MAXS];
  int max_iter;
  int n_rx;                        // surface reactions; the first is the one above, all n_rx in rxt
  int rate_area;                   // 1: rate scaled by the wall node's wetted area
  int halfway;                     // 1: wall placed half-way along each link
  real srcf[MAXS];                 // wall source factor: 1, or 1 / c_j (stoichiometric mass flux)
  int eq48;                        // 1: solid-gas coupling of Eq.(48) (else flux-matched)
  real kap[MAXS];                  // (D+2) / (2 Pr_j): gas conductivity per tau1_j C_j T / M_j
  // flow
  real F[3];
  real rho_in[MAXS], T_in, p_in;
  // 16-bit population storage: relative deviations g / rho_ref_j - wlat_i
  real rho_ref[MAXS], inv_rho_ref[MAXS];  // reference density per species
};

// lattice weights at rest and T = 1/3 (the equilibrium of Eq.(4) at u = 0):
// D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36
template <int D>
__host__ __device__ constexpr double wlat(int i) {
  return i == 0 ? (D == 2 ? 4.0 / 9.0 : 1.0 / 3.0)
                : (cnorm2<D>(i) == 1 ? (D == 2 ? 1.0 / 9.0 : 1.0 / 18.0) : 1.0 / 36.0);
}

// Population storage type PT: the arithmetic type itself (FP32, FP64) holds
// the populations; a 16-bit type (FP16, BF16) holds their relative deviations
// from the rest equilibrium at the reference density, g / rho_ref_j - wlat_i
// (O(0.01 - 1) for every species, inside FP16's normal range), in records
// padded to an even length (4-byte aligned).
template <typename PT>
__host__ __device__ constexpr bool narrow() {
  return sizeof(PT) == 2;
}
template <typename PT>
__host__ __device__ constexpr int rec_len(int ns) {
  return narrow<PT>() ? (ns + 1) / 2 * 2 : ns;
}

// Workspace pointers.  Populations and moments live in compact SLOT order:
// gas-like nodes in processing order (slot = gas-list index), then the wall
// nodes (slot = n_gas + wall index), then one null slot that no valid tap
// reads; slot_of maps a node to its slot (the null slot for interior solid).
// Populations are records of the NS species per (direction, slot), so one
// tap is one contiguous NS-value load for every species.
template <typename real, typename PT = real>
struct Bufs {
  PT *G[2];           // populations [((i*nsl + slot)*RL + j] (RL = rec_len(NS)), double-buffered
  PT *Gs;             // streamed (pre-collision) populations of the gas slots, same layout
  real *FR;           // per-slot record read by neighbours: u, T, rho_j, tau1_j
  real *FX;           // per-slot record of the node itself: tau2_j, u_j, U^c, energy defect
  real *Ts[2];        // solid temperature per node, double-buffered
  real *wall_r;       // molar rate per node (wall nodes) of the last step
  real *wall_q;       // reaction heat per wall node, last step (several reactions)
  const real *rxt;    // reaction table, RXS values per reaction (several reactions)
  real *wall_dE;      // kinetic energy the wall gave the gas, per node, last step
  real *cn_rhs, *cn_tmp;  // Crank-Nicolson solid: right-hand side and sweep buffer, per node
  const real *lj_tab;     // collision integrals: Omega_mu[lj_n] then Omega_D[lj_n]
  const uint8_t *kind;       // node class per node
  const int32_t *slot_of;    // slot per node
  const uint64_t *scls;      // streaming class word per gas/wall slot
  const uint32_t *wem;       // emission mask per wall node (wall order)
  const uint32_t *gas_list;  // node of each gas slot
  const uint32_t *wall_list; // node of each wall node
  double *acc_moles;  // per-block cumulative reaction extent
  double *acc_work;   // per-block cumulative body-force work
  double *acc_bheat;  // per-block cumulative Dirichlet-face heat
  double *acc_heat;   // per-block cumulative reaction heat (several reactions)
  double *partials;   // observe / residual reduction partials
  real *snap;         // residual snapshot per gas slot: X_j, T, u_a (sn_count values)
  real *snap_ts;      // residual snapshot of the solid temperature per node
  // stability record: [0] 1 once a gas node had a non-finite or negative
  // density or temperature, [1] the first such step (counted from 1 since
  // the last reset), [2] steps completed since the last reset
  int64_t *status;
};

// values per gas slot in the residual snapshot: mole fractions, T, u
__host__ __device__ constexpr int sn_count(int D, int ns) { return ns + 1 + D; }

// Field records per slot, grouped so that a kernel working on one species
// loads only that species' values.  FR (what the face neighbours' gradient
// stencils read): u_a, T, then (rho_j, tau1_j) pairs.  FX (read by the node
// itself): U^c_a, sum_j rho_j |u_j - u|^2, then (tau2_j, u_ja) groups of D+1.
__host__ __device__ constexpr int fr_u(int a) { return a; }
__host__ __device__ constexpr int fr_T(int D) { return D; }
__host__ __device__ constexpr int fr_rho(int D, int j) { return D + 1 + 2 * j; }
__host__ __device__ constexpr int fr_tau1(int D, int j) { return D + 2 + 2 * j; }
__host__ __device__ constexpr int fr_count(int D, int ns) { return D + 1 + 2 * ns; }
__host__ __device__ constexpr int fx_Uc(int a) { return a; }
__host__ __device__ constexpr int fx_ediff(int D) { return D; }
__host__ __device__ constexpr int fx_tau2(int D, int j) { return (D + 1) * (j + 1); }
__host__ __device__ constexpr int fx_uj(int D, int j, int a) { return (D + 1) * (j + 1) + 1 + a; }
__host__ __device__ constexpr int fx_count(int D, int ns) { return (D + 1) * (ns + 1); }

enum : uint8_t { KIND_GAS = 0, KIND_SOLID = 1, KIND_WALL = 2, KIND_INLET = 3, KIND_OUTLET = 4 };
__host__ __device__ inline bool gaslike(uint8_t k) { return k == KIND_GAS || k >= KIND_INLET; }

// ---------------------------------------------------------------------------
// Equilibrium of one species, Eq.(4) (mixture velocity) or Eq.(6) (species
// velocity): per axis the factors P0 = 1 - T - U^2, P+- = (T + U^2 +- U)/2
// with U = sqrt(M_j) u; D2Q9 takes their product, D3Q19 uses edges
// P_a P_b, faces P_a (1 - 2T - U_b^2 - U_c^2), and the rest the remainder.
// ---------------------------------------------------------------------------
template <typename real, int D>
__host__ __device__ inline void equilibrium(real rho, real sqM, const real *u, real T, real *f) {
  constexpr int Q = lat_q<D>();
  real U[3], U2[3], P0[3], Pp[3], Pm[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    U[a] = a < D ? sqM * u[a] : real(0);
    U2[a] = U[a] * U[a];
    P0[a] = real(1) - T - U2[a];
    Pp[a] = real(0.5) * (T + U2[a] + U[a]);
    Pm[a] = real(0.5) * (T + U2[a] - U[a]);
  }
  if (D == 2) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = cvec<D>(i, 0), cy = cvec<D>(i, 1);
      real fx = cx == 0 ? P0[0] : (cx > 0 ? Pp[0] : Pm[0]);
      real fy = cy == 0 ? P0[1] : (cy > 0 ? Pp[1] : Pm[1]);
      f[i] = rho * fx * fy;
    }
    return;
  }
  const real perp_base = real(1) - real(2) * T;
  real sum = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int c0 = cvec<D>(i, 0), c1 = cvec<D>(i, 1), c2 = cvec<D>(i, 2);
    const int nz = (c0 != 0) + (c1 != 0) + (c2 != 0);
    real v;
    if (nz == 1) {
      const int a = c0 != 0 ? 0 : (c1 != 0 ? 1 : 2);
      const int s = c0 + c1 + c2;
      real pa = s > 0 ? Pp[a] : Pm[a];
      real perp = perp_base;
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (b != a) perp -= U2[b];
      v = rho * pa * perp;
    } else {
      real prod = rho;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ca = cvec<D>(i, a);
        if (ca != 0) prod *= ca > 0 ? Pp[a] : Pm[a];
      }
      v = prod;
    }
    f[i] = v;
    sum += v;
  }
  f[0] = rho - sum;
}

// ---------------------------------------------------------------------------
// Source shapes (lattice velocities c_0i; species scaling applied by caller).
// psi_a: momentum only (Eq.(13) in 2-D): faces c_a, diagonals -c_a/4 (2-D)
//        or edges -c_a/8 (3-D).
// pi_aa: rest -1, faces along a +1/2.   pi_ab (a != b): c_a c_b / 4.
// chi_a: energy flux only: faces -c_a/2, diagonals c_a/4 (2-D), edges c_a/8.
// phi:   energy only: rest -1, faces 1/(2D).
// Each carries one moment of the lattice's natural moment basis and zero
// for all others.
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ constexpr bool is_face(int i) {
  return cnorm2<D>(i) == 1;
}

// k-th nonzero axis of direction i (k = 0, 1)
template <int D>
__host__ __device__ constexpr int edge_axis(int i, int k) {
  int seen = 0;
  for (int a = 0; a < 3; ++a)
    if (cvec<D>(i, a) != 0) {
      if (seen == k) return a;
      ++seen;
    }
  return 0;
}

}  // namespace fdlbm
