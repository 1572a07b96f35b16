// Host side of the C ABI declared in include/fdlbm.h: parameter validation,
// geometry pre-processing (node classes, streaming stencil classes, node
// lists), workspace layout, initial state, step scheduling, observables,
// field export and checkpoints.  All device work runs on the caller's stream.
#include "fdlbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "fdlbm_device.h"
#include "fdlbm_launch.h"

using namespace fdlbm;

namespace {
constexpr int NPROF = 4096;  // event pairs kept per kernel when profiling
}

struct fdlbm_ctx {
  fdlbm_desc d{};
  int D = 2, Q = 9, ns = 1, n = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // parameters (double on the host)
  double M[MAXS]{}, mu0[MAXS]{}, mu_T_exp = 0, Djk0[MAXS * MAXS]{}, D_T_exp = 0, D_p_exp = 0,
         T_ref = 1.0 / 3, p_ref = 1.0 / 3, Pr = 1;
  double Pr_j[MAXS] = {1, 1, 1, 1, 1, 1, 1, 1};  // per-species Prandtl numbers
  // Lennard-Jones transport: T_unit / eps_j, collision-integral table
  bool lj = false;
  int lj_n = 0;
  double lj_ie[MAXS]{}, lj_t0 = 0, lj_dt = 1, lj_om_mu[64]{}, lj_om_d[64]{};
  unsigned flags = FDLBM_CORR_ALL;
  double alpha_s = 0, C_s = 1, T_bc[6];
  int solid_scheme = FDLBM_SOLID_EULER;
  double nu[MAXS]{}, order[MAXS]{}, k0 = 0, ea = 0, T_ref_rxn = 1.0 / 3, dH = 0, T_iso = 1.0 / 3,
         tol = 1e-13;
  int wall_mode = 0, max_iter = 64;
  bool rate_area = false;  // rate per unit wetted wall area instead of per wall node
  bool source_flux = false;  // wall source nu_j M_j r / c_j (stoichiometric mass flux)
  bool halfway = false;      // wall half-way along each link instead of on the solid node
  // further surface reactions (fdlbm_add_reaction); reaction 0 is the one above
  int n_rx = 1;
  double xnu[MAXR][MAXS]{}, xord[MAXR][MAXS]{}, xk0[MAXR]{}, xea[MAXR]{}, xTref[MAXR]{}, xdH[MAXR]{};
  bool rx_set = false;
  int coupling = FDLBM_COUPLING_FLUX;  // solid-gas coupling at the wall nodes
  double F[3]{}, X_in[MAXS]{}, p_in = 1.0 / 3, T_in = 1.0 / 3;
  double rho_ref[MAXS]{};  // reference densities of 16-bit storage (mean initial density)
  bool species_set = false, geometry_set = false, bound = false, initialized = false;
  // geometry
  int inout = 0;
  std::vector<uint8_t> kind;
  std::vector<uint64_t> cls;       // class word per node (host only)
  std::vector<uint32_t> emask;     // emission mask per node (host only)
  std::vector<uint32_t> gas_list, wall_list;
  std::vector<int32_t> slot_of;    // slot per node (null slot for interior solid)
  std::vector<uint64_t> scls;      // class word per slot
  std::vector<uint32_t> wem;       // emission mask per wall node
  int64_t n_gas_fast = 0, n_wall_fast = 0;
  int64_t n_solid = 0;
  int nsl = 0;                     // slot stride
  int tile_rows = 0;               // y rows per tile of the processing order
  // workspace
  char *ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_cnr = 0, off_cnt = 0;  // Crank-Nicolson solid buffers
  size_t off_lj = 0;                // collision-integral table
  size_t off_rxt = 0, off_wq = 0, off_aq = 0;  // reaction table, heat per wall node, heat accumulator
  size_t off_G[2]{}, off_Gs = 0, off_FR = 0, off_FX = 0, off_Ts[2]{}, off_wr = 0, off_wde = 0, off_kind = 0, off_slot = 0,
         off_scls = 0, off_wem = 0, off_gl = 0, off_wl = 0, off_am = 0, off_aw = 0, off_ab = 0,
         off_part = 0, off_snap = 0, off_snapts = 0, off_status = 0;
  bool snap_valid = false;  // a residual snapshot exists
  int64_t snap_step = 0;    // step of the snapshot
  size_t total = 0;
  int acc_slots = 0, obs_blocks = 0;
  int cur = 0;
  int64_t step = 0;
  // stability record: its step count starts at status_base; with
  // check_every > 0 each fdlbm_step checks it after every check_every steps
  int64_t status_base = 0, check_every = 0, bad_step = -1;
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> events;  // [launch][kernel][2]
  int64_t prof_launches = 0;
  bool prof_recorded[K_NUM]{};  // kernel ids whose events the step records
  // second stream for the wall and solid kernels (created on the first step)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_wall = nullptr, ev_solid = nullptr;
  bool side_tried = false;
  bool overlap = true;  // use the second stream when it exists
};

static int set_err(fdlbm_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIPCHK(c, call)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return set_err(c, FDLBM_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static double wlat_of(int D, int i) { return D == 2 ? wlat<2>(i) : wlat<3>(i); }

// arithmetic type (moments, solid, wall arrays) and population storage type
static size_t real_size(const fdlbm_ctx *c) { return c->d.precision == FDLBM_F64 ? 8 : 4; }
static size_t pop_size(const fdlbm_ctx *c) {
  return c->d.precision == FDLBM_F64 ? 8 : (c->d.precision == FDLBM_F32 ? 4 : 2);
}
// values per population record (species, padded to an even count for 16-bit storage)
static int rec_count(const fdlbm_ctx *c) { return pop_size(c) == 2 ? (c->ns + 1) / 2 * 2 : c->ns; }

template <typename R, typename P>
struct PrecTag {
  using real = R;
  using pop = P;
};
// call fn(PrecTag<real, pop>{}) for the context's precision
template <typename Fn>
static int with_prec(const fdlbm_ctx *c, Fn &&fn) {
  switch (c->d.precision) {
    case FDLBM_F64: return fn(PrecTag<double, double>{});
    case FDLBM_F16: return fn(PrecTag<float, _Float16>{});
    case FDLBM_BF16: return fn(PrecTag<float, __bf16>{});
    default: return fn(PrecTag<float, float>{});
  }
}

// Workspace layout; depends on the geometry (slot counts).  Per-slot arrays
// have stride nsl = n_gas + n_wall + 1 rounded up to 64 (the +1 is the null
// slot of interior solid nodes).
static void layout(fdlbm_ctx *c) {
  const size_t b = real_size(c), n = (size_t)c->n;
  const size_t ng = c->gas_list.size(), nw = c->wall_list.size();
  c->nsl = (int)((ng + nw + 1 + 63) / 64 * 64);
  const size_t nsl = (size_t)c->nsl;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t pops = (size_t)rec_count(c) * c->Q * nsl * pop_size(c);
  c->off_G[0] = take(pops);
  c->off_G[1] = take(pops);
  c->off_Gs = take(pops);
  c->off_FR = take((size_t)fr_count(c->D, c->ns) * nsl * b);
  c->off_FX = take((size_t)fx_count(c->D, c->ns) * nsl * b);
  c->off_Ts[0] = take(n * b);
  c->off_Ts[1] = take(n * b);
  c->off_wr = take(n * b);
  c->off_wde = take(n * b);
  c->off_cnr = take(n * b);
  c->off_cnt = take(n * b);
  c->off_lj = take(128 * b);
  c->off_rxt = take((size_t)MAXR * RXS * b);
  c->off_wq = take(n * b);
  c->off_kind = take(n);
  c->off_slot = take(n * 4);
  c->off_scls = take(nsl * 8);
  c->off_wem = take(std::max<size_t>(nw, 1) * 4);
  c->off_gl = take(std::max<size_t>(ng, 1) * 4);
  c->off_wl = take(std::max<size_t>(nw, 1) * 4);
  // one accumulator slot per block of the largest grid that accumulates
  const int tiles = c->D == 2 ? solid_tiles<2>(c->d.nx, c->d.ny, c->d.nz)
                              : solid_tiles<3>(c->d.nx, c->d.ny, c->d.nz);
  c->acc_slots = std::max((int)((n + BLOCK - 1) / BLOCK) * c->ns, tiles) + 8 * c->ns + 8;
  c->off_am = take((size_t)c->acc_slots * 8);
  c->off_aw = take((size_t)c->acc_slots * 8);
  c->off_ab = take((size_t)c->acc_slots * 8);
  c->off_aq = take((size_t)c->acc_slots * 8);
  c->obs_blocks = 1024;
  c->off_part = take((size_t)c->obs_blocks * (MAXS + 9) * 8);
  c->off_snap = take((size_t)sn_count(c->D, c->ns) * nsl * b);
  c->off_snapts = take(n * b);
  c->off_status = take(4 * sizeof(int64_t));
  c->total = o;
}

template <typename real, typename PT>
static Bufs<real, PT> bufs(const fdlbm_ctx *c) {
  Bufs<real, PT> b;
  char *w = c->ws;
  b.G[0] = (PT *)(w + c->off_G[0]);
  b.G[1] = (PT *)(w + c->off_G[1]);
  b.Gs = (PT *)(w + c->off_Gs);
  b.FR = (real *)(w + c->off_FR);
  b.FX = (real *)(w + c->off_FX);
  b.Ts[0] = (real *)(w + c->off_Ts[0]);
  b.Ts[1] = (real *)(w + c->off_Ts[1]);
  b.wall_r = (real *)(w + c->off_wr);
  b.wall_dE = (real *)(w + c->off_wde);
  b.cn_rhs = (real *)(w + c->off_cnr);
  b.cn_tmp = (real *)(w + c->off_cnt);
  b.lj_tab = (const real *)(w + c->off_lj);
  b.rxt = (const real *)(w + c->off_rxt);
  b.wall_q = (real *)(w + c->off_wq);
  b.kind = (const uint8_t *)(w + c->off_kind);
  b.slot_of = (const int32_t *)(w + c->off_slot);
  b.scls = (const uint64_t *)(w + c->off_scls);
  b.wem = (const uint32_t *)(w + c->off_wem);
  b.gas_list = (const uint32_t *)(w + c->off_gl);
  b.wall_list = (const uint32_t *)(w + c->off_wl);
  b.acc_moles = (double *)(w + c->off_am);
  b.acc_work = (double *)(w + c->off_aw);
  b.acc_bheat = (double *)(w + c->off_ab);
  b.acc_heat = (double *)(w + c->off_aq);
  b.partials = (double *)(w + c->off_part);
  b.snap = (real *)(w + c->off_snap);
  b.snap_ts = (real *)(w + c->off_snapts);
  b.status = (int64_t *)(w + c->off_status);
  return b;
}

// Streaming weights of each stencil class at shift s (quadratic or degraded
// Lagrange interpolation through the class's taps), in the tap order of
// stencil_off().
static void class_weights(double s, double w[7][3]) {
  w[0][0] = 0.5 * s * (s - 1.0);
  w[0][1] = 1.0 - s * s;
  w[0][2] = 0.5 * s * (s + 1.0);
  w[1][0] = 0.5 * (1.0 - s) * (2.0 - s);
  w[1][1] = s * (2.0 - s);
  w[1][2] = 0.5 * s * (s - 1.0);
  w[2][0] = 0.5 * (1.0 + s) * (2.0 + s);
  w[2][1] = -s * (2.0 + s);
  w[2][2] = 0.5 * s * (1.0 + s);
  w[3][0] = 1.0 - s;
  w[3][1] = s;
  w[3][2] = 0;
  w[4][0] = -s;
  w[4][1] = 1.0 + s;
  w[4][2] = 0;
  w[5][0] = 1.0;
  w[5][1] = w[5][2] = 0;
  w[6][0] = 1.0;
  w[6][1] = w[6][2] = 0;
}

// collision integral from the table (the kernels' interpolation, in double)
static double lj_omega_host(const fdlbm_ctx *c, const double *om, double ts) {
  const double f = (ts - c->lj_t0) / c->lj_dt;
  if (!(f > 0.0)) return om[0];
  if (f >= c->lj_n - 1) return om[c->lj_n - 1];
  const int i = (int)f;
  const double w = f - i;
  return (1.0 - w) * om[i] + w * om[i + 1];
}

template <typename real>
static Params<real> params(const fdlbm_ctx *c) {
  Params<real> p;
  std::memset(&p, 0, sizeof p);
  p.ns = c->ns;
  p.nx = c->d.nx;
  p.ny = c->d.ny;
  p.nz = c->d.nz;
  p.n = c->n;
  for (int a = 0; a < 3; ++a) p.per[a] = c->d.periodic[a] ? 1 : 0;
  if (c->D == 2) p.per[2] = 1;
  p.inout = c->inout;
  p.flags = c->flags;
  p.wall_mode = c->wall_mode;
  p.n_gas = (int)c->gas_list.size();
  p.n_wall = (int)c->wall_list.size();
  p.nsl = c->nsl;
  p.n_gas_fast = (int)c->n_gas_fast;
  p.n_wall_fast = (int)c->n_wall_fast;
  p.slot_off_gas = (int)((c->n_gas_fast + BLOCK - 1) / BLOCK);
  p.slot_off_wall = (int)((c->n_wall_fast + BLOCK - 1) / BLOCK);
  for (int j = 0; j < c->ns; ++j) {
    const double cj = std::sqrt(1.0 / c->M[j]);
    p.M[j] = (real)c->M[j];
    p.invM[j] = (real)(1.0 / c->M[j]);
    p.sqM[j] = (real)std::sqrt(c->M[j]);
    p.cj[j] = (real)cj;
    p.cj2[j] = (real)(1.0 / c->M[j]);
    p.invcj[j] = (real)std::sqrt(c->M[j]);
    double w[7][3];
    class_weights(1.0 - cj, w);
    for (int k = 0; k < 7; ++k)
      for (int q = 0; q < 3; ++q) p.wint[j][k][q] = (real)w[k][q];
    p.mu0[j] = (real)c->mu0[j];
    p.nu[j] = (real)c->nu[j];
    p.srcf[j] = (real)(c->source_flux ? 1.0 / cj : 1.0);
    p.order[j] = (int)c->order[j];
    p.rho_in[j] = (real)(c->M[j] * c->X_in[j] * c->p_in / c->T_in);
  }
  // Wilke's phi_jk, Eq.(15) with the square of the bracket (phi_jj = 1); the
  // viscosity ratios are temperature independent (common exponent)
  for (int j = 0; j < c->ns; ++j)
    for (int k = 0; k < c->ns; ++k) {
      const double br = 1.0 + std::sqrt(c->mu0[j] / c->mu0[k]) * std::pow(c->M[k] / c->M[j], 0.25);
      p.wilke[j][k] = (real)(br * br / (std::sqrt(8.0) * std::sqrt(1.0 + c->M[j] / c->M[k])));
      p.invD0[j][k] = j == k ? real(0) : (real)(1.0 / c->Djk0[j * c->ns + k]);
    }
  p.mu_T_exp = (real)c->mu_T_exp;
  p.D_T_exp = (real)c->D_T_exp;
  p.D_p_exp = (real)c->D_p_exp;
  p.T_ref = (real)c->T_ref;
  p.p_ref = (real)c->p_ref;
  for (int j = 0; j < c->ns; ++j) p.kprj[j] = (real)((c->D + 2.0) * (1.0 / c->Pr_j[j] - 1.0));
  p.lj = c->lj ? 1 : 0;
  p.lj_n = c->lj_n;
  p.lj_t0 = (real)c->lj_t0;
  p.lj_idt = (real)(1.0 / c->lj_dt);
  if (c->lj) {
    // reference collision integrals folded into mu0 and 1/D0 (Eq.(26)-(27)
    // scaled from the reference state)
    for (int j = 0; j < c->ns; ++j) {
      p.lj_ie[j] = (real)c->lj_ie[j];
      p.mu0[j] = (real)(c->mu0[j] * lj_omega_host(c, c->lj_om_mu, c->T_ref * c->lj_ie[j]));
      for (int k = 0; k < c->ns; ++k)
        if (k != j)
          p.invD0[j][k] = (real)(1.0 / (c->Djk0[j * c->ns + k] *
                                        lj_omega_host(c, c->lj_om_d, c->T_ref * std::sqrt(c->lj_ie[j] * c->lj_ie[k]))));
    }
  }
  p.alpha_s = (real)c->alpha_s;
  p.C_s = (real)c->C_s;
  p.invCs = (real)(1.0 / c->C_s);
  // Crank-Nicolson: Jacobi sweeps from T contract the error by at most
  // rho = a D / (1 + a D) each (row sums of the iteration matrix), so enough
  // sweeps take it below the arithmetic's rounding relative to the step
  p.solid_cn = c->solid_scheme == FDLBM_SOLID_CN ? 1 : 0;
  p.eq48 = c->coupling == FDLBM_COUPLING_EQ48 ? 1 : 0;
  for (int j = 0; j < c->ns; ++j) p.kap[j] = (real)((c->D + 2.0) / (2.0 * c->Pr_j[j]));
  p.cn_iters = 0;
  if (p.solid_cn) {
    const double rho = c->alpha_s * c->D / (1.0 + c->alpha_s * c->D);
    const double tol = c->d.precision == FDLBM_F64 ? 1e-15 : 1e-8;
    p.cn_iters = rho > 0 ? (int)std::min(5000.0, std::ceil(std::log(tol) / std::log(rho))) : 1;
    p.cn_iters = std::max(p.cn_iters, 1);
  }
  for (int a = 0; a < 6; ++a) {
    p.has_bc[a] = !std::isnan(c->T_bc[a]);
    p.T_bc[a] = p.has_bc[a] ? (real)c->T_bc[a] : real(0);
  }
  p.k0 = (real)c->k0;
  p.ea = (real)c->ea;
  p.T_ref_rxn = (real)c->T_ref_rxn;
  p.dH = (real)c->dH;
  p.T_iso = (real)c->T_iso;
  p.tol = (real)std::max(c->tol, c->d.precision == FDLBM_F64 ? 0.0 : 4.0 * 1.1920929e-7);
  p.max_iter = c->max_iter;
  p.rate_area = c->rate_area ? 1 : 0;
  p.halfway = c->halfway ? 1 : 0;
  p.n_rx = c->n_rx;
  for (int a = 0; a < 3; ++a) p.F[a] = a < c->D ? (real)c->F[a] : real(0);
  p.T_in = (real)c->T_in;
  p.p_in = (real)c->p_in;
  for (int j = 0; j < c->ns; ++j) {
    p.rho_ref[j] = (real)c->rho_ref[j];
    p.inv_rho_ref[j] = (real)(1.0 / c->rho_ref[j]);
  }
  return p;
}

// ---------------------------------------------------------------------------
// geometry pre-processing
// ---------------------------------------------------------------------------
static void lattice_c(int D, int i, int *cv) {
  for (int a = 0; a < 3; ++a) cv[a] = D == 2 ? cvec<2>(i, a) : cvec<3>(i, a);
}

// node + k e_i, or -1 beyond a closed axis
static int shifted(const fdlbm_ctx *c, int node, int i, int k) {
  int cv[3];
  lattice_c(c->D, i, cv);
  const int lim[3] = {c->d.nx, c->d.ny, c->d.nz};
  int p[3] = {node % lim[0], (node / lim[0]) % lim[1], node / (lim[0] * lim[1])};
  for (int a = 0; a < 3; ++a) {
    p[a] += k * cv[a];
    if (p[a] < 0 || p[a] >= lim[a]) {
      const bool per = a == 2 && c->D == 2 ? true : c->d.periodic[a] != 0;
      if (!per) return -1;
      p[a] = ((p[a] % lim[a]) + lim[a]) % lim[a];
    }
  }
  return p[0] + lim[0] * (p[1] + lim[1] * p[2]);
}

int fdlbm_set_geometry(fdlbm_ctx *c, const uint8_t *mask, int inout) {
  if (!c || !mask) return set_err(c, FDLBM_E_INVALID, "null argument");
  if (c->bound) return set_err(c, FDLBM_E_STATE, "geometry must be set before binding the workspace");
  const int nx = c->d.nx, n = c->n, Q = c->Q;
  if (inout && (c->d.periodic[0] || nx < 6))
    return set_err(c, FDLBM_E_GEOMETRY, "inlet/outlet needs a closed x axis of at least 6 nodes");
  c->inout = inout ? 1 : 0;
  c->kind.assign(n, KIND_GAS);
  for (int node = 0; node < n; ++node) {
    const int x = node % nx;
    if (mask[node] > 1) return set_err(c, FDLBM_E_GEOMETRY, "mask values must be 0 or 1");
    const bool ghost_in = c->inout && x <= 1, ghost_out = c->inout && x >= nx - 2;
    if (mask[node] == 0) {
      c->kind[node] = ghost_in ? KIND_INLET : (ghost_out ? KIND_OUTLET : KIND_GAS);
    } else {
      if (ghost_in || ghost_out) return set_err(c, FDLBM_E_GEOMETRY, "inlet/outlet planes must be gas");
      c->kind[node] = KIND_SOLID;
    }
  }
  int64_t ngas = 0;
  for (int node = 0; node < n; ++node) {
    if (gaslike(c->kind[node])) {
      ++ngas;
      if (c->kind[node] == KIND_GAS)
        for (int i = 1; i < Q; ++i)
          if (shifted(c, node, i, 1) < 0)
            return set_err(c, FDLBM_E_GEOMETRY, "gas node %d touches a closed domain edge", node);
      continue;
    }
    for (int i = 1; i < Q; ++i) {
      const int y = shifted(c, node, i, 1);
      if (y >= 0 && gaslike(c->kind[y])) {
        c->kind[node] = KIND_WALL;
        break;
      }
    }
  }
  if (ngas == 0) return set_err(c, FDLBM_E_GEOMETRY, "no gas node");
  // an outlet node copies the collision of the last interior node of its row
  for (int node = 0; node < n; ++node)
    if (c->kind[node] == KIND_OUTLET && c->kind[node - node % nx + nx - 3] != KIND_GAS)
      return set_err(c, FDLBM_E_GEOMETRY, "outlet row of node %d has no gas node at x = nx - 3", node);
  // emission masks: gas emits along every direction, a wall node along the
  // directions that lead into the gas
  c->emask.assign(n, 0u);
  for (int node = 0; node < n; ++node) {
    const uint8_t k = c->kind[node];
    if (gaslike(k)) c->emask[node] = (1u << Q) - 1u;
    else if (k == KIND_WALL)
      for (int i = 1; i < Q; ++i) {
        const int y = shifted(c, node, i, 1);
        if (y >= 0 && gaslike(c->kind[y])) c->emask[node] |= 1u << i;
      }
  }
  auto emits = [&](int y, int i) { return y >= 0 && ((c->emask[y] >> i) & 1u); };
  // stencil class of each (destination, direction): the first of central,
  // forward, backward, two-point, two-point, one-point, one-point whose taps
  // all emit along the direction (Eq.(34)-(36) and their degraded forms)
  c->cls.assign(n, ~uint64_t(0));
  c->gas_list.clear();
  c->wall_list.clear();
  c->n_solid = 0;
  for (int node = 0; node < n; ++node) {
    const uint8_t k = c->kind[node];
    if (k == KIND_SOLID || k == KIND_WALL) ++c->n_solid;
    if (!(gaslike(k) || k == KIND_WALL)) continue;
    uint64_t w = 0;
    for (int i = 1; i < Q; ++i) {
      int cl = CLS_NONE;
      const bool dest = gaslike(k) || (k == KIND_WALL && [&] {
                          const int y = shifted(c, node, i, -1);
                          return y >= 0 && gaslike(c->kind[y]);
                        }());
      if (dest) {
        for (int cand = 0; cand < 7; ++cand) {
          bool ok = true;
          for (int q = 0; q < stencil_ntaps(cand) && ok; ++q)
            ok = emits(shifted(c, node, i, stencil_off(cand, q)), i);
          if (ok) {
            cl = cand;
            break;
          }
        }
        if (cl == CLS_NONE) return set_err(c, FDLBM_E_GEOMETRY, "no stencil at node %d", node);
      }
      w |= uint64_t(cl) << (3 * (i - 1));
    }
    c->cls[node] = w;
    if (gaslike(k)) c->gas_list.push_back((uint32_t)node);
    else c->wall_list.push_back((uint32_t)node);
  }
  // Processing (and slot) order: y-tiles of yt rows, within a tile z, then
  // y, then x.  A tap two planes upstream along z was then touched about
  // 2*yt*nx nodes earlier, a distance whose population traffic fits one
  // XCD's 4 MiB L2; in plain node order it would be two whole planes.
  {
    const double per_node = 2.0 * c->Q * rec_count(c) * (double)pop_size(c);
    int yt = 4;
    while (yt * 2 <= c->d.ny && 2.0 * c->d.nx * (yt * 2) * per_node <= 4.0 * 1048576.0) yt *= 2;
    if (c->D == 2) yt = c->d.ny;
    c->tile_rows = yt;
    const int nxx = c->d.nx, nyy = c->d.ny;
    auto key = [&](uint32_t node) {
      const int x = (int)(node % nxx), y = (int)((node / nxx) % nyy), z = (int)(node / ((uint32_t)nxx * nyy));
      return std::make_tuple(y / yt, z, y % yt, x);
    };
    auto by_tile = [&](uint32_t a, uint32_t b) { return key(a) < key(b); };
    std::stable_sort(c->gas_list.begin(), c->gas_list.end(), by_tile);
    std::stable_sort(c->wall_list.begin(), c->wall_list.end(), by_tile);
  }
  // then nodes whose taps (up to 3 nodes away) never wrap a periodic axis
  // first, so the kernels for them use plain strides
  auto no_wrap = [&](uint32_t node) {
    const int lim[3] = {c->d.nx, c->d.ny, c->d.nz};
    const int q[3] = {(int)(node % lim[0]), (int)((node / lim[0]) % lim[1]), (int)(node / (lim[0] * lim[1]))};
    for (int a = 0; a < c->D; ++a)
      if (c->d.periodic[a] && (q[a] < 3 || q[a] >= lim[a] - 3)) return false;
    return true;
  };
  auto split = [&](std::vector<uint32_t> &v) {
    auto mid = std::stable_partition(v.begin(), v.end(), no_wrap);
    return (int64_t)(mid - v.begin());
  };
  c->n_gas_fast = split(c->gas_list);
  c->n_wall_fast = split(c->wall_list);
  // slots: gas nodes in list order, then wall nodes, then the null slot
  const int ng = (int)c->gas_list.size(), nw = (int)c->wall_list.size();
  c->slot_of.assign(n, ng + nw);
  c->scls.assign((size_t)ng + nw, ~uint64_t(0));
  c->wem.assign((size_t)std::max(nw, 1), 0u);
  for (int t = 0; t < ng; ++t) {
    c->slot_of[c->gas_list[t]] = t;
    c->scls[t] = c->cls[c->gas_list[t]];
  }
  for (int w = 0; w < nw; ++w) {
    c->slot_of[c->wall_list[w]] = ng + w;
    c->scls[(size_t)ng + w] = c->cls[c->wall_list[w]];
    c->wem[w] = c->emask[c->wall_list[w]];
  }
  layout(c);
  // the population gathers use 32-bit byte offsets within one direction's
  // array: n_gas + n_wall slots of rec_count values each must stay below 4 GiB
  const double span = (double)c->nsl * rec_count(c) * (double)pop_size(c);
  if (span >= 4294967296.0)
    return set_err(c, FDLBM_E_INVALID,
                   "%zu gas and wall nodes: one direction's populations would take %.3g bytes, "
                   "more than the 4 GiB the kernels address",
                   c->gas_list.size() + c->wall_list.size(), span);
  c->geometry_set = true;
  return FDLBM_OK;
}

template <typename T>
static int copy_field(fdlbm_ctx *c, size_t off_bytes, size_t count, double *dst) {
  std::vector<T> tmp(count);
  HIPCHK(c, hipMemcpyAsync(tmp.data(), c->ws + off_bytes, count * sizeof(T), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t k = 0; k < count; ++k) {
    if constexpr (sizeof(T) == 8) dst[k] = (double)tmp[k];
    else dst[k] = (double)(float)tmp[k];  // 16-bit types convert through float
  }
  return FDLBM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// The public functions take C linkage from their declarations in fdlbm.h.

int fdlbm_create(const fdlbm_desc *d, fdlbm_ctx **out) {
  if (!d || !out) return FDLBM_E_INVALID;
  *out = nullptr;
  if ((d->lattice != FDLBM_D2Q9 && d->lattice != FDLBM_D3Q19) || d->nx < 1 || d->ny < 1 ||
      d->nz < 1 || (d->lattice == FDLBM_D2Q9 && d->nz != 1) || d->n_species < 1 ||
      d->n_species > MAX_NS || d->precision < FDLBM_F64 || d->precision > FDLBM_BF16)
    return FDLBM_E_INVALID;
  // node lookups (slot of a node, 4 bytes) use 32-bit byte offsets
  const double nn = (double)d->nx * d->ny * d->nz;
  if (nn > 1073741824.0) return FDLBM_E_INVALID;
  fdlbm_ctx *c = new fdlbm_ctx();
  c->d = *d;
  c->D = d->lattice;
  c->Q = d->lattice == FDLBM_D2Q9 ? 9 : 19;
  c->ns = d->n_species;
  c->n = d->nx * d->ny * d->nz;
  c->stream = (hipStream_t)d->hip_stream;
  for (int a = 0; a < 6; ++a) c->T_bc[a] = NAN;
  *out = c;
  return FDLBM_OK;
}

void fdlbm_destroy(fdlbm_ctx *c) {
  if (!c) return;
  for (auto &e : c->events) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  for (hipEvent_t e : {c->ev_fork, c->ev_wall, c->ev_solid})
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char *fdlbm_last_error(const fdlbm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int fdlbm_set_species(fdlbm_ctx *c, const double *M, const double *mu0, double mu_T_exp,
                      const double *Djk0, double D_T_exp, double D_p_exp, double T_ref,
                      double p_ref, double Pr, unsigned flags) {
  if (!c || !M || !mu0 || !Djk0) return set_err(c, FDLBM_E_INVALID, "null argument");
  for (int j = 0; j < c->ns; ++j) {
    if (!(M[j] >= 1.0) || !std::isfinite(M[j]))
      return set_err(c, FDLBM_E_INVALID, "masses are relative to the lightest species (>= 1)");
    if (!(mu0[j] > 0.0)) return set_err(c, FDLBM_E_INVALID, "viscosities must be positive");
    for (int k = 0; k < c->ns; ++k) {
      if (j != k && !(Djk0[j * c->ns + k] > 0.0))
        return set_err(c, FDLBM_E_INVALID, "binary diffusivities must be positive");
      if (j != k && Djk0[j * c->ns + k] != Djk0[k * c->ns + j])
        return set_err(c, FDLBM_E_INVALID, "binary diffusivities must be symmetric");
    }
  }
  if (!(T_ref > 0 && p_ref > 0 && Pr > 0)) return set_err(c, FDLBM_E_INVALID, "T_ref, p_ref, Pr must be positive");
  if (flags & ~FDLBM_CORR_ALL) return set_err(c, FDLBM_E_INVALID, "unknown correction flag");
  for (int j = 0; j < c->ns; ++j) {
    c->M[j] = M[j];
    c->mu0[j] = mu0[j];
    for (int k = 0; k < c->ns; ++k) c->Djk0[j * c->ns + k] = Djk0[j * c->ns + k];
  }
  c->mu_T_exp = mu_T_exp;
  c->D_T_exp = D_T_exp;
  c->D_p_exp = D_p_exp;
  c->T_ref = T_ref;
  c->p_ref = p_ref;
  c->Pr = Pr;
  for (int j = 0; j < MAXS; ++j) c->Pr_j[j] = Pr;
  c->flags = flags;
  c->species_set = true;
  return FDLBM_OK;
}

int fdlbm_set_prandtl(fdlbm_ctx *c, const double *Pr_j) {
  if (!c) return FDLBM_E_INVALID;
  if (!c->species_set) return set_err(c, FDLBM_E_STATE, "set the species first");
  for (int j = 0; j < c->ns; ++j) {
    const double v = Pr_j ? Pr_j[j] : c->Pr;
    if (!(v > 0)) return set_err(c, FDLBM_E_INVALID, "Prandtl numbers must be positive");
  }
  for (int j = 0; j < c->ns; ++j) c->Pr_j[j] = Pr_j ? Pr_j[j] : c->Pr;
  return FDLBM_OK;
}

int fdlbm_set_solid(fdlbm_ctx *c, double alpha_s, double C_s, const double *T_bc6) {
  if (!c) return FDLBM_E_INVALID;
  if (!(alpha_s >= 0.0)) return set_err(c, FDLBM_E_INVALID, "alpha_s must be non-negative");
  if (c->solid_scheme == FDLBM_SOLID_EULER && alpha_s > 0.5 / c->D)
    return set_err(c, FDLBM_E_INVALID, "alpha_s must lie in [0, 1/(2D)] (forward-Euler stability)");
  if (!(C_s > 0.0)) return set_err(c, FDLBM_E_INVALID, "C_s must be positive");
  c->alpha_s = alpha_s;
  c->C_s = C_s;
  for (int a = 0; a < 6; ++a) c->T_bc[a] = T_bc6 ? T_bc6[a] : NAN;
  return FDLBM_OK;
}

// the collision-integral table into the workspace, in the arithmetic type
static int upload_lj(fdlbm_ctx *c) {
  if (!c->bound || !c->lj) return FDLBM_OK;
  const size_t b = real_size(c);
  std::vector<char> buf(128 * b, 0);
  for (int i = 0; i < c->lj_n; ++i) {
    if (b == 8) {
      reinterpret_cast<double *>(buf.data())[i] = c->lj_om_mu[i];
      reinterpret_cast<double *>(buf.data())[c->lj_n + i] = c->lj_om_d[i];
    } else {
      reinterpret_cast<float *>(buf.data())[i] = (float)c->lj_om_mu[i];
      reinterpret_cast<float *>(buf.data())[c->lj_n + i] = (float)c->lj_om_d[i];
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_lj, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FDLBM_OK;
}

// the reaction table into the workspace, in the arithmetic type (reaction 0
// from fdlbm_set_reaction, the others from fdlbm_add_reaction)
static int upload_rx(fdlbm_ctx *c) {
  if (!c->bound || !c->rx_set) return FDLBM_OK;
  std::vector<double> t((size_t)MAXR * RXS, 0.0);
  for (int k = 0; k < c->n_rx; ++k) {
    double *r = &t[(size_t)k * RXS];
    r[RX_K0] = k ? c->xk0[k] : c->k0;
    r[RX_EA] = k ? c->xea[k] : c->ea;
    r[RX_TREF] = k ? c->xTref[k] : c->T_ref_rxn;
    r[RX_DH] = k ? c->xdH[k] : c->dH;
    for (int j = 0; j < c->ns; ++j) {
      r[RX_NU + j] = k ? c->xnu[k][j] : c->nu[j];
      r[RX_ORD + j] = k ? c->xord[k][j] : c->order[j];
    }
  }
  const size_t b = real_size(c);
  std::vector<char> buf(t.size() * b);
  for (size_t i = 0; i < t.size(); ++i) {
    if (b == 8) reinterpret_cast<double *>(buf.data())[i] = t[i];
    else reinterpret_cast<float *>(buf.data())[i] = (float)t[i];
  }
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_rxt, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FDLBM_OK;
}

int fdlbm_set_lj_transport(fdlbm_ctx *c, const double *eps_over_k, double T_unit, double tstar_min,
                           double tstar_max, int n, const double *omega_mu, const double *omega_d) {
  if (!c) return FDLBM_E_INVALID;
  if (!c->species_set) return set_err(c, FDLBM_E_STATE, "set the species first");
  if (!eps_over_k) {
    c->lj = false;
    return FDLBM_OK;
  }
  if (!omega_mu || !omega_d || n < 2 || n > 64 || !(tstar_max > tstar_min) || !(tstar_min > 0) ||
      !(T_unit > 0))
    return set_err(c, FDLBM_E_INVALID, "bad collision-integral table (2..64 points on tmin < tmax)");
  for (int i = 0; i < n; ++i)
    if (!(omega_mu[i] > 0 && omega_d[i] > 0)) return set_err(c, FDLBM_E_INVALID, "collision integrals must be positive");
  for (int j = 0; j < c->ns; ++j)
    if (!(eps_over_k[j] > 0)) return set_err(c, FDLBM_E_INVALID, "eps/k must be positive");
  for (int j = 0; j < c->ns; ++j) c->lj_ie[j] = T_unit / eps_over_k[j];
  c->lj_n = n;
  c->lj_t0 = tstar_min;
  c->lj_dt = (tstar_max - tstar_min) / (n - 1);
  for (int i = 0; i < n; ++i) {
    c->lj_om_mu[i] = omega_mu[i];
    c->lj_om_d[i] = omega_d[i];
  }
  c->lj = true;
  return upload_lj(c);
}

int fdlbm_set_solid_scheme(fdlbm_ctx *c, int scheme) {
  if (!c) return FDLBM_E_INVALID;
  if (scheme != FDLBM_SOLID_EULER && scheme != FDLBM_SOLID_CN)
    return set_err(c, FDLBM_E_INVALID, "unknown solid scheme %d", scheme);
  if (scheme == FDLBM_SOLID_EULER && c->alpha_s > 0.5 / c->D)
    return set_err(c, FDLBM_E_INVALID, "alpha_s > 1/(2D) needs the Crank-Nicolson scheme");
  if (scheme == FDLBM_SOLID_CN && c->coupling == FDLBM_COUPLING_EQ48)
    return set_err(c, FDLBM_E_INVALID, "the Eq.(48) coupling needs the forward-Euler solid");
  c->solid_scheme = scheme;
  return FDLBM_OK;
}

int fdlbm_set_reaction(fdlbm_ctx *c, const double *nu, const double *order, double k0, double ea,
                       double T_ref, double dH, int wall_mode, double T_iso, double tol,
                       int max_iter) {
  if (!c || !nu || !order) return set_err(c, FDLBM_E_INVALID, "null argument");
  for (int j = 0; j < c->ns; ++j)
    if (!(order[j] >= 0 && order[j] <= 3 && order[j] == std::floor(order[j])))
      return set_err(c, FDLBM_E_INVALID, "reaction orders must be integers 0..3");
  if (wall_mode != FDLBM_WALL_REACTIVE && wall_mode != FDLBM_WALL_ISOTHERMAL)
    return set_err(c, FDLBM_E_INVALID, "unknown wall mode");
  if (!(k0 >= 0) || !(T_ref > 0) || !(T_iso > 0) || max_iter < 0 || !(tol >= 0))
    return set_err(c, FDLBM_E_INVALID, "reaction parameters out of range");
  for (int j = 0; j < c->ns; ++j) {
    c->nu[j] = nu[j];
    c->order[j] = order[j];
  }
  c->k0 = k0;
  c->ea = ea;
  c->T_ref_rxn = T_ref;
  c->dH = dH;
  c->wall_mode = wall_mode;
  c->T_iso = T_iso;
  c->tol = tol;
  c->max_iter = max_iter;
  c->n_rx = 1;
  c->rx_set = true;
  return upload_rx(c);
}

int fdlbm_add_reaction(fdlbm_ctx *c, const double *nu, const double *order, double k0, double ea, double T_ref,
                       double dH) {
  if (!c || !nu || !order) return set_err(c, FDLBM_E_INVALID, "null argument");
  if (!c->rx_set) return set_err(c, FDLBM_E_STATE, "set the first reaction with fdlbm_set_reaction");
  if (c->n_rx >= MAXR) return set_err(c, FDLBM_E_INVALID, "at most %d surface reactions", MAXR);
  for (int j = 0; j < c->ns; ++j)
    if (!(order[j] >= 0 && order[j] <= 3 && order[j] == std::floor(order[j])))
      return set_err(c, FDLBM_E_INVALID, "reaction orders must be integers 0..3");
  if (!(k0 >= 0) || !(T_ref > 0)) return set_err(c, FDLBM_E_INVALID, "reaction parameters out of range");
  const int k = c->n_rx;
  for (int j = 0; j < c->ns; ++j) {
    c->xnu[k][j] = nu[j];
    c->xord[k][j] = order[j];
  }
  c->xk0[k] = k0;
  c->xea[k] = ea;
  c->xTref[k] = T_ref;
  c->xdH[k] = dH;
  c->n_rx = k + 1;
  return upload_rx(c);
}

int fdlbm_set_solid_coupling(fdlbm_ctx *c, int mode) {
  if (!c) return FDLBM_E_INVALID;
  if (mode != FDLBM_COUPLING_FLUX && mode != FDLBM_COUPLING_EQ48)
    return set_err(c, FDLBM_E_INVALID, "coupling must be FDLBM_COUPLING_FLUX or FDLBM_COUPLING_EQ48");
  if (mode == FDLBM_COUPLING_EQ48 && c->solid_scheme != FDLBM_SOLID_EULER)
    return set_err(c, FDLBM_E_INVALID, "the Eq.(48) coupling needs the forward-Euler solid");
  c->coupling = mode;
  return FDLBM_OK;
}

int fdlbm_set_rate_scaling(fdlbm_ctx *c, int mode) {
  if (!c) return FDLBM_E_INVALID;
  if (mode != FDLBM_RATE_PER_NODE && mode != FDLBM_RATE_PER_AREA)
    return set_err(c, FDLBM_E_INVALID, "rate scaling must be FDLBM_RATE_PER_NODE or FDLBM_RATE_PER_AREA");
  c->rate_area = mode == FDLBM_RATE_PER_AREA;
  return FDLBM_OK;
}

int fdlbm_set_wall_source(fdlbm_ctx *c, int mode) {
  if (!c) return FDLBM_E_INVALID;
  if (mode != FDLBM_SOURCE_LATTICE && mode != FDLBM_SOURCE_FLUX)
    return set_err(c, FDLBM_E_INVALID, "wall source must be FDLBM_SOURCE_LATTICE or FDLBM_SOURCE_FLUX");
  c->source_flux = mode == FDLBM_SOURCE_FLUX;
  return FDLBM_OK;
}

int fdlbm_set_wall_position(fdlbm_ctx *c, int position) {
  if (!c) return FDLBM_E_INVALID;
  if (position != FDLBM_WALL_ON_NODE && position != FDLBM_WALL_HALFWAY)
    return set_err(c, FDLBM_E_INVALID, "wall position must be FDLBM_WALL_ON_NODE or FDLBM_WALL_HALFWAY");
  c->halfway = position == FDLBM_WALL_HALFWAY;
  return FDLBM_OK;
}

int fdlbm_set_flow(fdlbm_ctx *c, const double *F3, const double *X_in, double p_in, double T_in) {
  if (!c) return FDLBM_E_INVALID;
  if (!(p_in > 0 && T_in > 0)) return set_err(c, FDLBM_E_INVALID, "inlet p and T must be positive");
  for (int a = 0; a < 3; ++a) c->F[a] = F3 ? F3[a] : 0.0;
  for (int j = 0; j < c->ns; ++j) c->X_in[j] = X_in ? X_in[j] : 0.0;
  c->p_in = p_in;
  c->T_in = T_in;
  return FDLBM_OK;
}

int fdlbm_workspace_bytes(const fdlbm_ctx *c, size_t *bytes) {
  if (!c || !bytes) return FDLBM_E_INVALID;
  if (!c->geometry_set) return FDLBM_E_STATE;
  *bytes = c->total;
  return FDLBM_OK;
}

int fdlbm_counts(const fdlbm_ctx *c, int64_t *ng, int64_t *nw, int64_t *ns) {
  if (!c || !c->geometry_set) return FDLBM_E_STATE;
  if (ng) *ng = (int64_t)c->gas_list.size();
  if (nw) *nw = (int64_t)c->wall_list.size();
  if (ns) *ns = c->n_solid;
  return FDLBM_OK;
}

int fdlbm_bind_workspace(fdlbm_ctx *c, void *dev, size_t bytes) {
  if (!c) return FDLBM_E_INVALID;
  if (!c->geometry_set) return set_err(c, FDLBM_E_STATE, "set the geometry before binding");
  if (!dev || ((uintptr_t)dev & 255u) || bytes < c->total)
    return set_err(c, FDLBM_E_ALIGN, "workspace must be >= %zu bytes and 256-byte aligned", c->total);
  c->ws = (char *)dev;
  c->ws_bytes = bytes;
  const size_t n = (size_t)c->n;
  HIPCHK(c, hipMemsetAsync(c->ws, 0, c->total, c->stream));
  auto up = [&](size_t off, const void *src, size_t bytes) {
    return bytes ? hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream) : hipSuccess;
  };
  HIPCHK(c, up(c->off_kind, c->kind.data(), n));
  HIPCHK(c, up(c->off_slot, c->slot_of.data(), n * 4));
  HIPCHK(c, up(c->off_scls, c->scls.data(), c->scls.size() * 8));
  HIPCHK(c, up(c->off_wem, c->wem.data(), c->wem.size() * 4));
  HIPCHK(c, up(c->off_gl, c->gas_list.data(), c->gas_list.size() * 4));
  HIPCHK(c, up(c->off_wl, c->wall_list.data(), c->wall_list.size() * 4));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->bound = true;
  c->initialized = false;
  const int rc = upload_lj(c);
  return rc != FDLBM_OK ? rc : upload_rx(c);
}

// clear the stability record (not inside any captured graph) and start its
// step count at the context's step
static int reset_status(fdlbm_ctx *c) {
  HIPCHK(c, hipMemsetAsync(c->ws + c->off_status, 0, 4 * sizeof(int64_t), c->stream));
  c->status_base = c->step;
  c->bad_step = -1;
  return FDLBM_OK;
}

// host-side equilibrium for the initial state (same closed form as the kernels)
template <typename real, typename PT>
static int init_impl(fdlbm_ctx *c, const double *rho, const double *u, const double *T,
                     const double *Ts) {
  const size_t n = (size_t)c->n, nsl = (size_t)c->nsl;
  const int Q = c->Q, ns = c->ns, RL = rec_count(c);
  // reference densities of 16-bit storage: mean initial density per species
  // (floored at 1e-12 of the mean total density so that it can be inverted)
  double tot = 0;
  for (int j = 0; j < ns; ++j) {
    double sum = 0;
    for (uint32_t node : c->gas_list) sum += rho[(size_t)j * n + node];
    c->rho_ref[j] = sum / (double)c->gas_list.size();
    tot += c->rho_ref[j];
  }
  for (int j = 0; j < ns; ++j) c->rho_ref[j] = std::max(c->rho_ref[j], 1e-12 * tot);
  const Params<real> pr = params<real>(c);
  std::vector<PT> G((size_t)RL * Q * nsl, PT(0.0f));
  std::vector<real> hT(n, real(0));
  // moment records of the gas slots before the first step (the half-way
  // wall reads their velocity and temperature); the wall slots' records are
  // written by every step's wall kernel
  const int NR = fr_count(c->D, ns);
  std::vector<real> FRh((size_t)NR * nsl, real(0));
  auto put = [&](int i, size_t slot, int j, real v) {
    if (narrow<PT>()) v = v * pr.inv_rho_ref[j] - real(wlat_of(c->D, i));  // as the kernels do
    G[((size_t)i * nsl + slot) * RL + j] = PT(v);
  };
  for (size_t node = 0; node < n; ++node) {
    hT[node] = (real)Ts[node];
    if (!gaslike(c->kind[node])) continue;
    const size_t slot = (size_t)c->slot_of[node];
    real uu[3] = {(real)u[node], (real)u[n + node], (real)u[2 * n + node]};
    for (int a = 0; a < c->D; ++a) FRh[slot * NR + fr_u(a)] = uu[a];
    FRh[slot * NR + fr_T(c->D)] = (real)T[node];
    for (int j = 0; j < ns; ++j) FRh[slot * NR + fr_rho(c->D, j)] = (real)rho[j * n + node];
    for (int j = 0; j < ns; ++j) {
      real f[19];
      const real sq = (real)std::sqrt(c->M[j]);
      if (c->D == 2) equilibrium<real, 2>((real)rho[j * n + node], sq, uu, (real)T[node], f);
      else equilibrium<real, 3>((real)rho[j * n + node], sq, uu, (real)T[node], f);
      for (int i = 0; i < Q; ++i) put(i, slot, j, f[i]);
    }
  }
  for (size_t node = 0; node < n; ++node) {
    if (c->kind[node] != KIND_WALL) continue;
    const real Tw = c->wall_mode == FDLBM_WALL_ISOTHERMAL ? (real)c->T_iso : (real)Ts[node];
    real wt[19];
    const real u0[3] = {0, 0, 0};
    if (c->D == 2) equilibrium<real, 2>(real(1), real(1), u0, Tw, wt);
    else equilibrium<real, 3>(real(1), real(1), u0, Tw, wt);
    for (int j = 0; j < ns; ++j) {
      double sum = 0;
      int cnt = 0;
      for (int i = 1; i < Q; ++i) {
        const int y = shifted(c, (int)node, i, 1);
        if (y >= 0 && gaslike(c->kind[y])) {
          sum += rho[j * n + y];
          ++cnt;
        }
      }
      const real rw = (real)(sum / cnt);
      for (int i = 1; i < Q; ++i)
        if ((c->emask[node] >> i) & 1u) put(i, (size_t)c->slot_of[node], j, rw * wt[i]);
    }
  }
  c->cur = 0;
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_G[0], G.data(), G.size() * sizeof(PT),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_FR, FRh.data(), FRh.size() * sizeof(real), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_Ts[0], hT.data(), n * sizeof(real), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_Ts[1], hT.data(), n * sizeof(real), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemsetAsync(c->ws + c->off_am, 0, (size_t)c->acc_slots * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->ws + c->off_aw, 0, (size_t)c->acc_slots * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->ws + c->off_ab, 0, (size_t)c->acc_slots * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->ws + c->off_aq, 0, (size_t)c->acc_slots * 8, c->stream));
  c->step = 0;
  if (reset_status(c) != FDLBM_OK) return FDLBM_E_HIP;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->initialized = true;
  c->snap_valid = false;
  return FDLBM_OK;
}

int fdlbm_init_fields(fdlbm_ctx *c, const double *rho, const double *u, const double *T,
                      const double *Ts) {
  if (!c) return FDLBM_E_INVALID;
  if (!c->bound || !c->species_set) return set_err(c, FDLBM_E_STATE, "bind the workspace and set species first");
  if (!rho || !u || !T || !Ts) return set_err(c, FDLBM_E_INVALID, "null argument");
  return with_prec(c, [&](auto tag) {
    using Tg = decltype(tag);
    return init_impl<typename Tg::real, typename Tg::pop>(c, rho, u, T, Ts);
  });
}

int fdlbm_set_profiling(fdlbm_ctx *c, int enable) {
  if (!c) return FDLBM_E_INVALID;
  if (enable && c->events.empty()) {
    c->events.resize((size_t)NPROF * K_NUM * 2);
    for (auto &e : c->events) HIPCHK(c, hipEventCreate(&e));
  }
  c->prof = enable != 0;
  c->prof_launches = 0;
  return FDLBM_OK;
}

int fdlbm_kernel_times(fdlbm_ctx *c, double *avg_ms, int64_t *launches) {
  if (!c || !avg_ms) return FDLBM_E_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int64_t L = std::min<int64_t>(c->prof_launches, NPROF);
  for (int k = 0; k < K_NUM; ++k) {
    double tot = 0;
    int64_t cnt = 0;
    for (int64_t l = 0; l < L && c->prof_recorded[k]; ++l) {
      hipEvent_t a = c->events[((size_t)l * K_NUM + k) * 2], b = c->events[((size_t)l * K_NUM + k) * 2 + 1];
      float ms = 0;
      if (hipEventQuery(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess) {
        tot += ms;
        ++cnt;
      }
    }
    avg_ms[k] = cnt ? tot / cnt : 0.0;
  }
  (void)hipGetLastError();  // event queries must not leave a sticky error behind
  if (launches) *launches = L;
  return FDLBM_OK;
}

template <typename real, typename PT>
static int step_impl(fdlbm_ctx *c, int64_t n_steps) {
  const Params<real> pr = params<real>(c);
  const Bufs<real, PT> bu = bufs<real, PT>(c);
  if (!c->side_tried) {
    // a non-blocking second stream at the default priority, ordered against
    // the context's stream by events only; without it the step runs on one
    c->side_tried = true;
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_wall, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_solid, hipEventDisableTiming) != hipSuccess) {
      if (c->side) (void)hipStreamDestroy(c->side);
      c->side = nullptr;
      (void)hipGetLastError();
    }
  }
  for (int64_t s = 0; s < n_steps; ++s) {
    LaunchInfo li;
    li.stream = c->stream;
    li.n_solid = (int)c->n_solid;
    li.side = c->overlap ? c->side : nullptr;
    li.ev_fork = c->ev_fork;
    li.ev_wall = c->ev_wall;
    li.ev_solid = c->ev_solid;
    li.events = nullptr;
    for (int k = 0; k < K_NUM; ++k) li.recorded[k] = false;
    if (c->prof && c->prof_launches < NPROF)
      li.events = &c->events[(size_t)c->prof_launches * K_NUM * 2];
    hipError_t e = launch_step<real, PT>(c->D, pr, bu, c->cur, li);
    if (e != hipSuccess) return set_err(c, FDLBM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    if (li.events) {
      ++c->prof_launches;
      for (int k = 0; k < K_NUM; ++k) c->prof_recorded[k] = li.recorded[k];
    }
    c->cur ^= 1;
    ++c->step;
  }
  return FDLBM_OK;
}

// read the stability record (synchronises the stream): the first unstable
// step, counted like fdlbm_obs.step, or -1
static int read_status(fdlbm_ctx *c, int64_t *first_bad) {
  int64_t st[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(st, c->ws + c->off_status, sizeof st, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *first_bad = st[0] ? c->status_base + st[1] : -1;
  return FDLBM_OK;
}

int fdlbm_step(fdlbm_ctx *c, int64_t n_steps) {
  if (!c) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "initialise the fields first");
  if (n_steps < 0) return set_err(c, FDLBM_E_INVALID, "negative step count");
  auto run = [&](int64_t k) {
    return with_prec(c, [&](auto tag) {
      using Tg = decltype(tag);
      return step_impl<typename Tg::real, typename Tg::pop>(c, k);
    });
  };
  if (c->check_every <= 0) return run(n_steps);
  // checked mode: chunks of check_every steps, stopping after the chunk in
  // which the stability record was set
  for (int64_t done = 0; done < n_steps;) {
    const int64_t k = std::min(c->check_every, n_steps - done);
    int rc = run(k);
    if (rc != FDLBM_OK) return rc;
    done += k;
    int64_t bad = -1;
    rc = read_status(c, &bad);
    if (rc != FDLBM_OK) return rc;
    if (bad >= 0) {
      c->bad_step = bad;
      return set_err(c, FDLBM_E_UNSTABLE,
                     "non-finite or negative density or temperature first seen in step %lld "
                     "(stopped after step %lld)", (long long)bad, (long long)c->step);
    }
  }
  return FDLBM_OK;
}

int fdlbm_set_sync_check(fdlbm_ctx *c, int64_t every) {
  if (!c) return FDLBM_E_INVALID;
  if (every < 0) return set_err(c, FDLBM_E_INVALID, "negative check interval");
  c->check_every = every;
  return FDLBM_OK;
}

int fdlbm_last_step(fdlbm_ctx *c, int64_t *step) {
  if (!c || !step) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "initialise the fields first");
  int64_t bad = -1;
  const int rc = read_status(c, &bad);
  if (rc != FDLBM_OK) return rc;
  *step = bad;
  return FDLBM_OK;
}

int fdlbm_set_overlap(fdlbm_ctx *c, int enable) {
  if (!c) return FDLBM_E_INVALID;
  c->overlap = enable != 0;
  return FDLBM_OK;
}

int fdlbm_sync(fdlbm_ctx *c) {
  if (!c) return FDLBM_E_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FDLBM_OK;
}

int fdlbm_observe(fdlbm_ctx *c, fdlbm_obs *o) {
  if (!c || !o) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "initialise the fields first");
  const hipError_t e = (hipError_t)with_prec(c, [&](auto tag) {
    using Tg = decltype(tag);
    using real = typename Tg::real;
    using PT = typename Tg::pop;
    return (int)launch_observe<real, PT>(c->D, params<real>(c), bufs<real, PT>(c), c->cur, c->obs_blocks,
                                         c->stream);
  });
  if (e != hipSuccess) return set_err(c, FDLBM_E_HIP, "observe launch: %s", hipGetErrorString(e));
  const int NP = c->ns + 9;
  std::vector<double> part((size_t)c->obs_blocks * NP);
  std::vector<double> acc(4 * (size_t)c->acc_slots);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->ws + c->off_part, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(acc.data(), c->ws + c->off_am, (size_t)c->acc_slots * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(acc.data() + c->acc_slots, c->ws + c->off_aw, (size_t)c->acc_slots * 8,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(acc.data() + 2 * c->acc_slots, c->ws + c->off_ab, (size_t)c->acc_slots * 8,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(acc.data() + 3 * c->acc_slots, c->ws + c->off_aq, (size_t)c->acc_slots * 8,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memset(o, 0, sizeof *o);
  const int ns = c->ns;
  o->T_min = o->rho_min = o->Ts_min = 1e300;
  o->T_max = o->Ts_max = -1e300;
  for (int bk = 0; bk < c->obs_blocks; ++bk) {
    const double *q = &part[(size_t)bk * NP];
    for (int j = 0; j < ns; ++j) o->mass[j] += q[j];
    o->e_gas += q[ns];
    o->e_solid += q[ns + 1];
    o->T_min = std::min(o->T_min, q[ns + 2]);
    o->T_max = std::max(o->T_max, q[ns + 3]);
    o->u_max = std::max(o->u_max, q[ns + 4]);
    o->rho_min = std::min(o->rho_min, q[ns + 5]);
    o->Ts_min = std::min(o->Ts_min, q[ns + 6]);
    o->Ts_max = std::max(o->Ts_max, q[ns + 7]);
    if (q[ns + 8] != 0.0) o->bad = 1;
  }
  double heat = 0.0;
  for (int s = 0; s < c->acc_slots; ++s) {
    o->moles_reacted += acc[s];
    o->work_body += acc[c->acc_slots + s];
    o->heat_boundary += acc[2 * c->acc_slots + s];
    heat += acc[3 * c->acc_slots + s];
  }
  // one reaction: its enthalpy times the moles; several: their heat summed per wall node
  o->heat_released = c->n_rx == 1 ? -c->dH * o->moles_reacted : heat;
  if (o->rho_min < 0) o->bad = 1;
  o->step = c->step;
  o->n_gas = (int32_t)c->gas_list.size();
  o->n_wall = (int32_t)c->wall_list.size();
  o->n_solid = (int32_t)c->n_solid;
  return FDLBM_OK;
}

// ---------------------------------------------------------------------------
// fdlbm_observe_noalloc: the observables with every scratch value in a
// file-scope device array instead of the workspace and host vectors.  The
// observe kernel writes its per-block partial sums there (every block
// overwrites its row, so nothing needs clearing), k_obs_fold folds them in
// the host's order, and the host copies the folded values into a stack
// array.  Each GPU holds its own copy of the array until the process ends;
// its device address is looked up once per device.
// ---------------------------------------------------------------------------
namespace {
constexpr int OBS_BLOCKS = 1024;                       // grid of the observe kernel
constexpr int OBS_FOLD = MAXS + 9 + 4;                 // folded values: partial slots + 4 sums
constexpr size_t SCRATCH_DOUBLES = (size_t)OBS_BLOCKS * (MAXS + 9) + 64;  // 139,776 bytes
constexpr int MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

// Fold the per-block partials (blocks rows of np values at part) and the
// four accumulator arrays (acc_slots each) exactly as fdlbm_observe does on
// the host: sums in block order, minima and maxima by the same comparisons,
// so the results are bitwise those of fdlbm_observe.  One thread per value.
__global__ void k_obs_fold(const double *part, int blocks, int ns, const double *am, const double *aw,
                           const double *ab, const double *aq, int acc_slots, double *out) {
  const int k = threadIdx.x, np = ns + 9;
  if (k < np) {
    const bool is_min = k == ns + 2 || k == ns + 5 || k == ns + 6;
    const bool is_max = k == ns + 3 || k == ns + 4 || k == ns + 7;
    double v = is_min ? 1e300 : (k == ns + 3 || k == ns + 7 ? -1e300 : 0.0);
    for (int bk = 0; bk < blocks; ++bk) {
      const double q = part[(size_t)bk * np + k];
      if (is_min) v = q < v ? q : v;
      else if (is_max) v = v < q ? q : v;
      else if (k == ns + 8) v = (q != 0.0) ? 1.0 : v;
      else v += q;
    }
    out[k] = v;
  } else if (k < np + 4) {
    const double *a = k == np ? am : (k == np + 1 ? aw : (k == np + 2 ? ab : aq));
    double v = 0.0;
    for (int s = 0; s < acc_slots; ++s) v += a[s];
    out[k] = v;
  }
}

// device address of this GPU's scratch array (looked up on the first call)
static int scratch_ptr(fdlbm_ctx *c, double **ptr) {
  static void *addr[MAX_DEVICES] = {};
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return set_err(c, FDLBM_E_INVALID, "device %d out of range", dev);
  if (!addr[dev]) {
    void *a = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    addr[dev] = a;
  }
  *ptr = (double *)addr[dev];
  return FDLBM_OK;
}

int fdlbm_observe_noalloc(fdlbm_ctx *c, fdlbm_obs *o) {
  if (!c || !o) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "initialise the fields first");
  const int ns = c->ns, NP = ns + 9;
  if ((size_t)c->obs_blocks * NP + OBS_FOLD > SCRATCH_DOUBLES || c->obs_blocks > OBS_BLOCKS)
    return set_err(c, FDLBM_E_INVALID, "observe needs %zu scratch values, the static array holds %zu",
                   (size_t)c->obs_blocks * NP + OBS_FOLD, SCRATCH_DOUBLES);
  double *sp = nullptr;
  const int rc = scratch_ptr(c, &sp);
  if (rc != FDLBM_OK) return rc;
  double *part = sp, *fold = sp + (size_t)c->obs_blocks * NP;
  const hipError_t e = (hipError_t)with_prec(c, [&](auto tag) {
    using Tg = decltype(tag);
    using real = typename Tg::real;
    using PT = typename Tg::pop;
    Bufs<real, PT> bu = bufs<real, PT>(c);
    bu.partials = part;  // the kernel's partial sums go to the static array
    return (int)launch_observe<real, PT>(c->D, params<real>(c), bu, c->cur, c->obs_blocks, c->stream);
  });
  if (e != hipSuccess) return set_err(c, FDLBM_E_HIP, "observe launch: %s", hipGetErrorString(e));
  hipLaunchKernelGGL(k_obs_fold, dim3(1), dim3(64), 0, c->stream, (const double *)part, c->obs_blocks, ns,
                     (const double *)(c->ws + c->off_am), (const double *)(c->ws + c->off_aw),
                     (const double *)(c->ws + c->off_ab), (const double *)(c->ws + c->off_aq), c->acc_slots,
                     fold);
  HIPCHK(c, hipGetLastError());
  double v[OBS_FOLD];
  HIPCHK(c, hipMemcpyAsync(v, fold, (size_t)(NP + 4) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memset(o, 0, sizeof *o);
  for (int j = 0; j < ns; ++j) o->mass[j] = v[j];
  o->e_gas = v[ns];
  o->e_solid = v[ns + 1];
  o->T_min = v[ns + 2];
  o->T_max = v[ns + 3];
  o->u_max = v[ns + 4];
  o->rho_min = v[ns + 5];
  o->Ts_min = v[ns + 6];
  o->Ts_max = v[ns + 7];
  o->bad = v[ns + 8] != 0.0 ? 1 : 0;
  o->moles_reacted = v[NP];
  o->work_body = v[NP + 1];
  o->heat_boundary = v[NP + 2];
  o->heat_released = c->n_rx == 1 ? -c->dH * o->moles_reacted : v[NP + 3];
  if (o->rho_min < 0) o->bad = 1;
  o->step = c->step;
  o->n_gas = (int32_t)c->gas_list.size();
  o->n_wall = (int32_t)c->wall_list.size();
  o->n_solid = (int32_t)c->n_solid;
  return FDLBM_OK;
}

int fdlbm_residual(fdlbm_ctx *c, double *r5) {
  if (!c || !r5) return FDLBM_E_INVALID;
  if (!c->initialized || c->step == 0) return set_err(c, FDLBM_E_STATE, "the residual needs a completed step");
  const hipError_t e = (hipError_t)with_prec(c, [&](auto tag) {
    using Tg = decltype(tag);
    using real = typename Tg::real;
    using PT = typename Tg::pop;
    return (int)launch_residual<real, PT>(c->D, params<real>(c), bufs<real, PT>(c), c->cur, c->obs_blocks,
                                          c->stream);
  });
  if (e != hipSuccess) return set_err(c, FDLBM_E_HIP, "residual launch: %s", hipGetErrorString(e));
  std::vector<double> part((size_t)c->obs_blocks * 8);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->ws + c->off_part, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double sums[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int bk = 0; bk < c->obs_blocks; ++bk)
    for (int k = 0; k < 8; ++k) sums[k] += part[(size_t)bk * 8 + k];
  const double K = (double)(c->step - c->snap_step);
  double rmax = 0;
  for (int g = 0; g < 4; ++g) {
    double r;
    if (!c->snap_valid || K <= 0) r = HUGE_VAL;
    else if (sums[2 * g] == 0.0) r = 0.0;
    else r = sums[2 * g + 1] > 0.0 ? std::sqrt(sums[2 * g]) / (K * std::sqrt(sums[2 * g + 1])) : HUGE_VAL;
    r5[g] = r;
    rmax = std::max(rmax, r);
  }
  r5[4] = rmax;
  c->snap_valid = true;
  c->snap_step = c->step;
  return FDLBM_OK;
}

int fdlbm_get_field(fdlbm_ctx *c, int field, int comp, double *dst) {
  if (!c || !dst) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "initialise the fields first");
  const size_t n = (size_t)c->n, b = real_size(c);
  const bool f64 = c->d.precision == FDLBM_F64;
  auto cp = [&](size_t off, size_t count) {
    return f64 ? copy_field<double>(c, off, count, dst) : copy_field<float>(c, off, count, dst);
  };
  int rc = FDLBM_OK;
  switch (field) {
    case FDLBM_FIELD_RHO:
    case FDLBM_FIELD_U:
    case FDLBM_FIELD_T: {
      if (c->step == 0) return set_err(c, FDLBM_E_STATE, "moments exist after the first step");
      int k;
      if (field == FDLBM_FIELD_RHO) {
        if (comp < 0 || comp >= c->ns) return set_err(c, FDLBM_E_INVALID, "bad species");
        k = fr_rho(c->D, comp);
      } else if (field == FDLBM_FIELD_U) {
        if (comp < 0 || comp > 2) return set_err(c, FDLBM_E_INVALID, "bad axis");
        if (comp >= c->D) {
          std::fill(dst, dst + n, 0.0);
          return FDLBM_OK;
        }
        k = fr_u(comp);
      } else {
        k = fr_T(c->D);
      }
      const size_t NR = (size_t)fr_count(c->D, c->ns);
      std::vector<double> v((size_t)c->nsl * NR);
      rc = f64 ? copy_field<double>(c, c->off_FR, v.size(), v.data())
               : copy_field<float>(c, c->off_FR, v.size(), v.data());
      if (rc) return rc;
      for (size_t x = 0; x < n; ++x)
        dst[x] = (gaslike(c->kind[x]) || c->kind[x] == KIND_WALL) ? v[(size_t)c->slot_of[x] * NR + k] : 0.0;
      return FDLBM_OK;
    }
    case FDLBM_FIELD_X: {
      if (c->step == 0) return set_err(c, FDLBM_E_STATE, "moments exist after the first step");
      if (comp < 0 || comp >= c->ns) return set_err(c, FDLBM_E_INVALID, "bad species");
      const size_t NR = (size_t)fr_count(c->D, c->ns);
      std::vector<double> v((size_t)c->nsl * NR);
      rc = f64 ? copy_field<double>(c, c->off_FR, v.size(), v.data())
               : copy_field<float>(c, c->off_FR, v.size(), v.data());
      if (rc) return rc;
      for (size_t x = 0; x < n; ++x) {
        // the same arithmetic as the device copy (fdlbm_get_field_device)
#pragma clang fp contract(off)
        dst[x] = 0.0;
        if (!(gaslike(c->kind[x]) || c->kind[x] == KIND_WALL)) continue;
        const double *r = &v[(size_t)c->slot_of[x] * NR];
        double C = 0.0;
        for (int j = 0; j < c->ns; ++j) C += r[fr_rho(c->D, j)] * (1.0 / c->M[j]);
        dst[x] = C > 0.0 ? r[fr_rho(c->D, comp)] * (1.0 / c->M[comp]) / C : 0.0;
      }
      return FDLBM_OK;
    }
    case FDLBM_FIELD_TS:
      rc = cp(c->off_Ts[c->cur], n);
      if (rc) return rc;
      for (size_t x = 0; x < n; ++x)
        if (!(c->kind[x] == KIND_SOLID || c->kind[x] == KIND_WALL)) dst[x] = 0.0;
      return FDLBM_OK;
    case FDLBM_FIELD_POP: {
      if (comp < 0 || comp >= c->ns) return set_err(c, FDLBM_E_INVALID, "bad species");
      const size_t nsl = (size_t)c->nsl, null_slot = c->gas_list.size() + c->wall_list.size();
      const size_t RL = (size_t)rec_count(c);
      std::vector<double> v((size_t)c->Q * nsl * RL);
      rc = with_prec(c, [&](auto tag) {
        using PT = typename decltype(tag)::pop;
        return copy_field<PT>(c, c->off_G[c->cur], v.size(), v.data());
      });
      if (rc) return rc;
      // 16-bit storage holds g / rho_ref_j - wlat_i (decoded in FP32, as the kernels);
      // a wall node stores nothing on the directions it does not emit along
      const bool dev = pop_size(c) == 2;
      const size_t ng = c->gas_list.size();
      const float rref = (float)c->rho_ref[comp];
      for (int i = 0; i < c->Q; ++i) {
        const float wl = (float)wlat_of(c->D, i);
        for (size_t x = 0; x < n; ++x) {
          const size_t sl = (size_t)c->slot_of[x];
          const bool stored = sl < ng || (sl < null_slot && ((c->wem[sl - ng] >> i) & 1u));
          const double raw = stored ? v[((size_t)i * nsl + sl) * RL + comp] : 0.0;
          dst[(size_t)i * n + x] = !stored ? 0.0 : (dev ? (double)(((float)raw + wl) * rref) : raw);
        }
      }
      return FDLBM_OK;
    }
    case FDLBM_FIELD_KIND:
      for (size_t x = 0; x < n; ++x) dst[x] = c->kind[x];
      return FDLBM_OK;
    case FDLBM_FIELD_WALL_R:
    case FDLBM_FIELD_WALL_DE:
      if (c->step == 0) return set_err(c, FDLBM_E_STATE, "wall values exist after the first step");
      rc = cp(field == FDLBM_FIELD_WALL_R ? c->off_wr : c->off_wde, n);
      if (rc) return rc;
      for (size_t x = 0; x < n; ++x)
        if (c->kind[x] != KIND_WALL) dst[x] = 0.0;
      return FDLBM_OK;
  }
  return set_err(c, FDLBM_E_INVALID, "unknown field");
}

// Fields into a device buffer (node order, FP64): a gather from the slot
// records, or a masked copy of a node-ordered array.
namespace {
constexpr int FIELD_BLOCK = 256;
struct InvM {
  double v[MAXS];
};
// mode 0: record entry k; 1: mole fraction of species k; 2: zero
template <typename real>
__global__ void __launch_bounds__(FIELD_BLOCK) k_field_rec(const real *__restrict__ FR, int NR, int mode, int k,
                                                          int D, int ns, InvM im,
                                                          const int32_t *__restrict__ slot_of,
                                                          const uint8_t *__restrict__ kind, int n,
                                                          double *__restrict__ dst) {
  const int x = blockIdx.x * FIELD_BLOCK + threadIdx.x;
  if (x >= n) return;
  const uint8_t kd = kind[x];
  double v = 0.0;
  if (mode != 2 && (gaslike(kd) || kd == KIND_WALL)) {
    const real *r = FR + (size_t)slot_of[x] * NR;
    if (mode == 0) {
      v = (double)r[k];
    } else {
      // no fused multiply-add: the host copy rounds each product
#pragma clang fp contract(off)
      double C = 0.0;
      for (int j = 0; j < ns; ++j) C += (double)r[fr_rho(D, j)] * im.v[j];
      v = C > 0.0 ? (double)r[fr_rho(D, k)] * im.v[k] / C : 0.0;
    }
  }
  dst[x] = v;
}
// mode 0: solid and wall nodes; 1: wall nodes; 2: every node (a byte array)
template <typename real>
__global__ void __launch_bounds__(FIELD_BLOCK) k_field_node(const real *__restrict__ a,
                                                           const uint8_t *__restrict__ bytes, int mode,
                                                           const uint8_t *__restrict__ kind, int n,
                                                           double *__restrict__ dst) {
  const int x = blockIdx.x * FIELD_BLOCK + threadIdx.x;
  if (x >= n) return;
  const uint8_t kd = kind[x];
  double v;
  if (mode == 2) v = (double)bytes[x];
  else if (mode == 1) v = kd == KIND_WALL ? (double)a[x] : 0.0;
  else v = (kd == KIND_SOLID || kd == KIND_WALL) ? (double)a[x] : 0.0;
  dst[x] = v;
}
}  // namespace

template <typename real>
static int field_device(fdlbm_ctx *c, int field, int comp, double *dst) {
  const int n = (int)c->n;
  const dim3 grid((unsigned)((n + FIELD_BLOCK - 1) / FIELD_BLOCK)), blk(FIELD_BLOCK);
  const real *FR = reinterpret_cast<const real *>(c->ws + c->off_FR);
  const int32_t *so = reinterpret_cast<const int32_t *>(c->ws + c->off_slot);
  const uint8_t *kind = reinterpret_cast<const uint8_t *>(c->ws + c->off_kind);
  const int NR = fr_count(c->D, c->ns);
  InvM im{};
  for (int j = 0; j < c->ns; ++j) im.v[j] = 1.0 / c->M[j];
  switch (field) {
    case FDLBM_FIELD_RHO:
    case FDLBM_FIELD_X:
    case FDLBM_FIELD_U:
    case FDLBM_FIELD_T: {
      int mode = 0, k = 0;
      if (field == FDLBM_FIELD_RHO || field == FDLBM_FIELD_X) {
        if (comp < 0 || comp >= c->ns) return set_err(c, FDLBM_E_INVALID, "bad species");
        mode = field == FDLBM_FIELD_X ? 1 : 0;
        k = field == FDLBM_FIELD_X ? comp : fr_rho(c->D, comp);
      } else if (field == FDLBM_FIELD_U) {
        if (comp < 0 || comp > 2) return set_err(c, FDLBM_E_INVALID, "bad axis");
        mode = comp >= c->D ? 2 : 0;
        k = comp >= c->D ? 0 : fr_u(comp);
      } else {
        k = fr_T(c->D);
      }
      hipLaunchKernelGGL(k_field_rec<real>, grid, blk, 0, c->stream, FR, NR, mode, k, c->D, c->ns, im, so,
                         kind, n, dst);
      break;
    }
    case FDLBM_FIELD_TS:
    case FDLBM_FIELD_WALL_R:
    case FDLBM_FIELD_WALL_DE: {
      const size_t off = field == FDLBM_FIELD_TS ? c->off_Ts[c->cur] : field == FDLBM_FIELD_WALL_R ? c->off_wr : c->off_wde;
      hipLaunchKernelGGL(k_field_node<real>, grid, blk, 0, c->stream, reinterpret_cast<const real *>(c->ws + off),
                         nullptr, field == FDLBM_FIELD_TS ? 0 : 1, kind, n, dst);
      break;
    }
    case FDLBM_FIELD_KIND:
      hipLaunchKernelGGL(k_field_node<real>, grid, blk, 0, c->stream, nullptr, kind, 2, kind, n, dst);
      break;
    default:
      return set_err(c, FDLBM_E_INVALID, "field not available on the device");
  }
  HIPCHK(c, hipGetLastError());
  return FDLBM_OK;
}

int fdlbm_get_field_device(fdlbm_ctx *c, int field, int comp, double *dst_device) {
  if (!c || !dst_device) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "initialise the fields first");
  if (c->step == 0 && field != FDLBM_FIELD_TS && field != FDLBM_FIELD_KIND)
    return set_err(c, FDLBM_E_STATE, "moments and wall values exist after the first step");
  return c->d.precision == FDLBM_F64 ? field_device<double>(c, field, comp, dst_device)
                                     : field_device<float>(c, field, comp, dst_device);
}

// checkpoint: header, populations (current buffer), solid temperature,
// per-step wall arrays, moments, accumulators
struct StateHeader {
  uint64_t magic, total, step;
  int32_t cur, pad;
  double rho_ref[MAXS];  // reference densities of 16-bit population storage
};

int fdlbm_state_bytes(const fdlbm_ctx *c, size_t *bytes) {
  if (!c || !bytes) return FDLBM_E_INVALID;
  *bytes = sizeof(StateHeader) + c->total;
  return FDLBM_OK;
}

int fdlbm_save_state(fdlbm_ctx *c, void *host, size_t bytes) {
  if (!c || !host) return FDLBM_E_INVALID;
  if (!c->initialized) return set_err(c, FDLBM_E_STATE, "nothing to save");
  if (bytes < sizeof(StateHeader) + c->total) return set_err(c, FDLBM_E_INVALID, "buffer too small");
  StateHeader h{0x46444c424d535432ull, c->total, (uint64_t)c->step, c->cur, 0, {}};
  for (int j = 0; j < MAXS; ++j) h.rho_ref[j] = c->rho_ref[j];
  std::memcpy(host, &h, sizeof h);
  HIPCHK(c, hipMemcpyAsync((char *)host + sizeof h, c->ws, c->total, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FDLBM_OK;
}

int fdlbm_load_state(fdlbm_ctx *c, const void *host, size_t bytes) {
  if (!c || !host) return FDLBM_E_INVALID;
  if (!c->bound) return set_err(c, FDLBM_E_STATE, "bind the workspace first");
  StateHeader h;
  if (bytes < sizeof h) return set_err(c, FDLBM_E_INVALID, "buffer too small");
  std::memcpy(&h, host, sizeof h);
  if (h.magic != 0x46444c424d535432ull || h.total != c->total || bytes < sizeof h + c->total)
    return set_err(c, FDLBM_E_INVALID, "state does not match this context");
  HIPCHK(c, hipMemcpyAsync(c->ws, (const char *)host + sizeof h, c->total, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->step = (int64_t)h.step;
  c->cur = h.cur;
  for (int j = 0; j < MAXS; ++j) c->rho_ref[j] = h.rho_ref[j];
  if (reset_status(c) != FDLBM_OK) return FDLBM_E_HIP;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->snap_valid = false;
  c->initialized = true;
  return FDLBM_OK;
}


// ---------------------------------------------------------------------------
// batches: many contexts advanced by shared persistent launches
// ---------------------------------------------------------------------------
struct fdlbm_batch {
  std::vector<fdlbm_ctx *> ctx;
  int n = 0, D = 3, ns = 1, precision = FDLBM_F32;
  hipStream_t stream = nullptr;
  std::string err;
  char *ws = nullptr;
  size_t ws_bytes = 0, total = 0;
  size_t p_size = 0, b_size = 0;
  size_t off_params = 0, off_bufs = 0, off_count = 0, off_items[BL_NUM]{};
  int max_items[BL_NUM]{};
  int n_items[BL_NUM]{};
  int grid[BL_NUM]{};
  std::vector<uint8_t> active;
  std::vector<char> h_params, h_bufs;        // host images (kept alive for async uploads)
  std::vector<int2> h_items[BL_NUM];
  int h_count[BL_NUM]{};
  int cur = 0;                               // parity the kernels are launched with
  int graph_steps = 20;
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // one per starting parity
  bool bound = false;
  // second stream for the wall and solid launches of a full step
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_wall = nullptr, ev_solid = nullptr;
  bool overlap = true;
  bool halfway = false, multi = false;  // wall variants, the same in every sample
  bool eq48 = false;                    // Eq.(48) coupling in every sample
  bool cn = false;                      // Crank-Nicolson solid in every sample
  int cn_iters = 0;                     // the largest sample's Jacobi sweeps (at the last upload)
};

static int bset_err(fdlbm_batch *b, int code, const char *fmt, ...) {
  if (b) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
  }
  return code;
}

#define BHIPCHK(b, call)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return bset_err(b, FDLBM_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static void batch_drop_graphs(fdlbm_batch *b) {
  for (auto &e : b->exec) {
    if (e) (void)hipGraphExecDestroy(e);
    e = nullptr;
  }
}

// logical blocks of each launch kind for one context
static void batch_blocks(const fdlbm_ctx *c, int nbk[BL_NUM]) {
  auto nb = [](int64_t cnt) { return (int)((cnt + BLOCK - 1) / BLOCK); };
  const int64_t ng = (int64_t)c->gas_list.size(), nw = (int64_t)c->wall_list.size();
  nbk[BL_WALL_FAST] = nb(c->n_wall_fast);
  nbk[BL_WALL_SLOW] = nb(nw - c->n_wall_fast);
  nbk[BL_GAS_FAST] = nb(c->n_gas_fast);
  nbk[BL_GAS_SLOW] = nb(ng - c->n_gas_fast);
  nbk[BL_COLLIDE] = nb(ng);
  nbk[BL_SOLID] = c->n_solid > 0 ? (c->D == 2 ? solid_tiles<2>(c->d.nx, c->d.ny, c->d.nz)
                                              : solid_tiles<3>(c->d.nx, c->d.ny, c->d.nz))
                                 : 0;
}

static int round8(int v) { return (v + 7) / 8 * 8; }

int fdlbm_batch_create(fdlbm_ctx *const *ctxs, int n, fdlbm_batch **out) {
  if (!out) return FDLBM_E_INVALID;
  *out = nullptr;
  if (!ctxs || n <= 0 || n > 65536) return FDLBM_E_INVALID;
  auto *b = new fdlbm_batch;
  b->n = n;
  b->ctx.assign(ctxs, ctxs + n);
  auto fail = [&](const char *msg) {
    if (ctxs[0]) set_err(ctxs[0], FDLBM_E_INVALID, "batch: %s", msg);
    delete b;
    return FDLBM_E_INVALID;
  };
  for (int s = 0; s < n; ++s) {
    const fdlbm_ctx *c = ctxs[s];
    if (!c) return fail("null context");
    if (!c->initialized) return fail("every context needs initialised fields");
    if (c->solid_scheme != ctxs[0]->solid_scheme) return fail("samples differ in the solid scheme");
    if (c->coupling != ctxs[0]->coupling) return fail("samples differ in the solid-gas coupling");
    if (c->halfway != ctxs[0]->halfway || (c->n_rx > 1) != (ctxs[0]->n_rx > 1))
      return fail("samples differ in the wall position or in having several surface reactions");
    if (c->D != ctxs[0]->D || c->ns != ctxs[0]->ns || c->d.precision != ctxs[0]->d.precision ||
        c->stream != ctxs[0]->stream)
      return fail("contexts differ in lattice, species count, precision or stream");
    for (int r = 0; r < s; ++r)
      if (ctxs[r] == c) return fail("a context appears twice");
  }
  b->D = ctxs[0]->D;
  b->ns = ctxs[0]->ns;
  b->halfway = ctxs[0]->halfway;
  b->multi = ctxs[0]->n_rx > 1;
  b->eq48 = ctxs[0]->coupling == FDLBM_COUPLING_EQ48;
  b->cn = ctxs[0]->solid_scheme == FDLBM_SOLID_CN;
  b->precision = ctxs[0]->d.precision;
  b->stream = ctxs[0]->stream;
  b->cur = ctxs[0]->cur;
  b->active.assign(n, 1);
  with_prec(ctxs[0], [&](auto tag) {
    using Tg = decltype(tag);
    b->p_size = sizeof(Params<typename Tg::real>);
    b->b_size = sizeof(Bufs<typename Tg::real, typename Tg::pop>);
    return 0;
  });
  for (int s = 0; s < n; ++s) {
    int nbk[BL_NUM];
    batch_blocks(ctxs[s], nbk);
    for (int k = 0; k < BL_NUM; ++k) b->max_items[k] += nbk[k];
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  b->off_params = take(b->p_size * n);
  b->off_bufs = take(b->b_size * n);
  b->off_count = take(sizeof(int) * BL_NUM);
  for (int k = 0; k < BL_NUM; ++k) b->off_items[k] = take(sizeof(int2) * std::max(1, b->max_items[k]));
  b->total = off;
  // default persistent grids: every logical block its own workgroup up to
  // 8 per CU (256 CUs), a multiple of the 8 XCDs
  for (int k = 0; k < BL_NUM; ++k) b->grid[k] = round8(std::min(b->max_items[k], 2048));
  // a non-blocking second stream at the default priority (ordered by events
  // only); without it the batched steps run on one stream
  if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_wall, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_solid, hipEventDisableTiming) != hipSuccess) {
    if (b->side) (void)hipStreamDestroy(b->side);
    b->side = nullptr;
    (void)hipGetLastError();
  }
  *out = b;
  return FDLBM_OK;
}

void fdlbm_batch_destroy(fdlbm_batch *b) {
  if (!b) return;
  batch_drop_graphs(b);
  if (b->side) {
    (void)hipStreamSynchronize(b->side);
    (void)hipStreamDestroy(b->side);
  }
  for (hipEvent_t e : {b->ev_fork, b->ev_wall, b->ev_solid})
    if (e) (void)hipEventDestroy(e);
  delete b;
}

const char *fdlbm_batch_last_error(const fdlbm_batch *b) { return b ? b->err.c_str() : "null batch"; }

int fdlbm_batch_workspace_bytes(const fdlbm_batch *b, size_t *bytes) {
  if (!b || !bytes) return FDLBM_E_INVALID;
  *bytes = b->total;
  return FDLBM_OK;
}

// Upload per-sample parameters, buffer tables (with each sample's population
// and solid-temperature buffers swapped where its parity differs from the
// batch's) and the work lists of the active samples; synchronous.
static int batch_upload(fdlbm_batch *b) {
  // the launch variants are the batch's: a member changed since creation
  // (wall position, several reactions, coupling, solid scheme) is refused
  for (int s = 0; s < b->n; ++s) {
    const fdlbm_ctx *c = b->ctx[s];
    if (c->halfway != b->halfway || (c->n_rx > 1) != b->multi ||
        (c->coupling == FDLBM_COUPLING_EQ48) != b->eq48 || (c->solid_scheme == FDLBM_SOLID_CN) != b->cn)
      return bset_err(b, FDLBM_E_INVALID,
                      "sample %d changed its wall position, reaction count, coupling or solid scheme "
                      "after the batch was created", s);
  }
  b->h_params.assign(b->p_size * b->n, 0);
  b->h_bufs.assign(b->b_size * b->n, 0);
  const int cn_before = b->cn_iters;  // graphs hold the sweep count they were captured with
  b->cn_iters = 0;
  for (int s = 0; s < b->n; ++s) {
    const fdlbm_ctx *c = b->ctx[s];
    const bool flip = (c->cur ^ b->cur) != 0;
    with_prec(c, [&](auto tag) {
      using Tg = decltype(tag);
      using real = typename Tg::real;
      using PT = typename Tg::pop;
      const Params<real> p = params<real>(c);
      Bufs<real, PT> bu = bufs<real, PT>(c);
      if (flip) {
        std::swap(bu.G[0], bu.G[1]);
        std::swap(bu.Ts[0], bu.Ts[1]);
      }
      std::memcpy(b->h_params.data() + b->p_size * s, &p, sizeof p);
      std::memcpy(b->h_bufs.data() + b->b_size * s, &bu, sizeof bu);
      b->cn_iters = std::max(b->cn_iters, p.cn_iters);
      return 0;
    });
  }
  if (b->cn_iters != cn_before) batch_drop_graphs(b);
  for (int k = 0; k < BL_NUM; ++k) b->h_items[k].clear();
  for (int s = 0; s < b->n; ++s) {
    if (!b->active[s]) continue;
    int nbk[BL_NUM];
    batch_blocks(b->ctx[s], nbk);
    for (int k = 0; k < BL_NUM; ++k)
      for (int q = 0; q < nbk[k]; ++q) b->h_items[k].push_back(make_int2(s, q));
  }
  for (int k = 0; k < BL_NUM; ++k) {
    b->n_items[k] = b->h_count[k] = (int)b->h_items[k].size();
    if (b->n_items[k])
      BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_items[k], b->h_items[k].data(), b->h_items[k].size() * sizeof(int2),
                                hipMemcpyHostToDevice, b->stream));
  }
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_params, b->h_params.data(), b->h_params.size(), hipMemcpyHostToDevice,
                            b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_bufs, b->h_bufs.data(), b->h_bufs.size(), hipMemcpyHostToDevice,
                            b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_count, b->h_count, sizeof b->h_count, hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  return FDLBM_OK;
}

int fdlbm_batch_bind_workspace(fdlbm_batch *b, void *dev, size_t bytes) {
  if (!b) return FDLBM_E_INVALID;
  if (!dev || ((uintptr_t)dev & 255u) || bytes < b->total)
    return bset_err(b, FDLBM_E_ALIGN, "batch workspace must be >= %zu bytes and 256-byte aligned", b->total);
  batch_drop_graphs(b);
  b->ws = (char *)dev;
  b->ws_bytes = bytes;
  const int rc = batch_upload(b);
  if (rc != FDLBM_OK) return rc;
  b->bound = true;
  return FDLBM_OK;
}

int fdlbm_batch_set_active(fdlbm_batch *b, const uint8_t *active) {
  if (!b || !active) return FDLBM_E_INVALID;
  if (!b->bound) return bset_err(b, FDLBM_E_STATE, "bind the batch workspace first");
  for (int s = 0; s < b->n; ++s) b->active[s] = active[s] ? 1 : 0;
  return batch_upload(b);
}

int fdlbm_batch_set_grid(fdlbm_batch *b, const int *grid, int graph_steps) {
  if (!b) return FDLBM_E_INVALID;
  if (grid)
    for (int k = 0; k < BL_NUM; ++k) {
      if (grid[k] <= 0 || grid[k] % 8) return bset_err(b, FDLBM_E_INVALID, "grids are positive multiples of 8");
    }
  if (graph_steps < 0 || graph_steps % 2) return bset_err(b, FDLBM_E_INVALID, "graph steps: even and >= 0");
  if (grid)
    for (int k = 0; k < BL_NUM; ++k) b->grid[k] = grid[k];
  if (graph_steps > 0) b->graph_steps = graph_steps;
  batch_drop_graphs(b);
  return FDLBM_OK;
}

int fdlbm_batch_set_overlap(fdlbm_batch *b, int enable) {
  if (!b) return FDLBM_E_INVALID;
  b->overlap = enable != 0;
  batch_drop_graphs(b);
  return FDLBM_OK;
}

int fdlbm_batch_get_grid(const fdlbm_batch *b, int *grid, int *graph_steps) {
  if (!b) return FDLBM_E_INVALID;
  if (grid)
    for (int k = 0; k < BL_NUM; ++k) grid[k] = b->grid[k];
  if (graph_steps) *graph_steps = b->graph_steps;
  return FDLBM_OK;
}

// one step of the kinds in `mask` (bit k = launch kind k) at parity cur
static hipError_t batch_launch(fdlbm_batch *b, int cur, unsigned mask) {
  BatchLaunch bl;
  bl.params = b->ws + b->off_params;
  bl.bufs = b->ws + b->off_bufs;
  for (int k = 0; k < BL_NUM; ++k) {
    bl.items[k] = (const int2 *)(b->ws + b->off_items[k]);
    bl.max_items[k] = b->max_items[k];
    bl.grid[k] = ((mask >> k) & 1u) ? std::min(b->grid[k], std::max(8, round8(b->max_items[k]))) : 0;
  }
  bl.count = (const int *)(b->ws + b->off_count);
  bl.stream = b->stream;
  // the second stream only for whole steps (the autotuner times single kinds)
  const bool whole = mask == (1u << BL_NUM) - 1;
  bl.side = whole && b->overlap ? b->side : nullptr;
  bl.ev_fork = b->ev_fork;
  bl.ev_wall = b->ev_wall;
  bl.ev_solid = b->ev_solid;
  bl.halfway = b->halfway ? 1 : 0;
  bl.multi = b->multi ? 1 : 0;
  bl.eq48 = b->eq48 ? 1 : 0;
  bl.cn_iters = b->cn ? b->cn_iters : 0;
  return (hipError_t)with_prec(b->ctx[0], [&](auto tag) {
    using Tg = decltype(tag);
    return (int)launch_batch_step<typename Tg::real, typename Tg::pop>(b->D, b->ns, bl, cur);
  });
}

static void batch_advance(fdlbm_batch *b, int64_t steps) {
  for (int s = 0; s < b->n; ++s)
    if (b->active[s]) {
      b->ctx[s]->step += steps;
      b->ctx[s]->cur ^= (int)(steps & 1);
    }
  b->cur ^= (int)(steps & 1);
}

static int batch_capture(fdlbm_batch *b, int parity) {
  hipGraph_t g = nullptr;
  BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < b->graph_steps && e == hipSuccess; ++k) e = batch_launch(b, parity ^ (k & 1), (1u << BL_NUM) - 1);
  const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bset_err(b, FDLBM_E_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&b->exec[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->exec[parity] = nullptr;
    return bset_err(b, FDLBM_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
  }
  return FDLBM_OK;
}

int fdlbm_batch_step(fdlbm_batch *b, int64_t n_steps) {
  if (!b) return FDLBM_E_INVALID;
  if (!b->bound) return bset_err(b, FDLBM_E_STATE, "bind the batch workspace first");
  if (n_steps < 0) return bset_err(b, FDLBM_E_INVALID, "negative step count");
  bool any = false;
  for (int s = 0; s < b->n; ++s) any = any || b->active[s];
  if (!any || n_steps == 0) return FDLBM_OK;
  // the legacy default stream cannot be captured: direct launches only there
  while (b->stream != nullptr && n_steps >= b->graph_steps) {
    if (!b->exec[b->cur]) {
      const int rc = batch_capture(b, b->cur);
      if (rc != FDLBM_OK) return rc;
    }
    BHIPCHK(b, hipGraphLaunch(b->exec[b->cur], b->stream));
    batch_advance(b, b->graph_steps);  // even: parity unchanged
    n_steps -= b->graph_steps;
  }
  for (; n_steps > 0; --n_steps) {
    const hipError_t e = batch_launch(b, b->cur, (1u << BL_NUM) - 1);
    if (e != hipSuccess) return bset_err(b, FDLBM_E_HIP, "batch launch: %s", hipGetErrorString(e));
    batch_advance(b, 1);
  }
  return FDLBM_OK;
}

int fdlbm_batch_check(fdlbm_batch *b, int *sample, int64_t *step) {
  if (!b || !sample || !step) return FDLBM_E_INVALID;
  if (!b->bound) return bset_err(b, FDLBM_E_STATE, "bind the batch workspace first");
  *sample = -1;
  *step = -1;
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  for (int s = 0; s < b->n; ++s) {
    int64_t bad = -1;
    if (read_status(b->ctx[s], &bad) != FDLBM_OK)
      return bset_err(b, FDLBM_E_HIP, "sample %d: %s", s, b->ctx[s]->err.c_str());
    if (bad >= 0) {
      *sample = s;
      *step = bad;
      return bset_err(b, FDLBM_E_UNSTABLE,
                      "sample %d: non-finite or negative density or temperature first seen in step %lld", s,
                      (long long)bad);
    }
  }
  return FDLBM_OK;
}

// Autotuner of the persistent launch shapes: for each candidate grid size
// (workgroups per launch, a multiple of 8) every launch kind is timed with
// HIP events over `steps` steps (after one warm-up step), and each kind keeps
// its fastest grid.  The tuning steps are real steps of the active samples.
int fdlbm_batch_autotune(fdlbm_batch *b, int steps, int *grid_out) {
  if (!b) return FDLBM_E_INVALID;
  if (!b->bound) return bset_err(b, FDLBM_E_STATE, "bind the batch workspace first");
  if (steps <= 0 || steps > 10000) return bset_err(b, FDLBM_E_INVALID, "steps in 1..10000");
  static const int cand[] = {256, 512, 1024, 2048, 4096, 8192, 16384};
  const int ncand = (int)(sizeof cand / sizeof cand[0]);
  std::vector<hipEvent_t> ev((size_t)BL_NUM * 2);
  for (auto &e : ev) BHIPCHK(b, hipEventCreate(&e));
  double best_t[BL_NUM];
  int best_g[BL_NUM];
  const int saved[BL_NUM] = {b->grid[0], b->grid[1], b->grid[2], b->grid[3], b->grid[4], b->grid[5]};
  for (int k = 0; k < BL_NUM; ++k) {
    best_t[k] = HUGE_VAL;
    best_g[k] = saved[k];
  }
  int rc = FDLBM_OK;
  int maxcap = 8;
  for (int k = 0; k < BL_NUM; ++k) maxcap = std::max(maxcap, round8(b->max_items[k]));
  // candidates up to the first one that gives every kind all its blocks
  for (int ci = 0; ci < ncand && rc == FDLBM_OK && (ci == 0 || cand[ci - 1] < maxcap); ++ci) {
    for (int k = 0; k < BL_NUM; ++k) b->grid[k] = std::min(cand[ci], std::max(8, round8(b->max_items[k])));
    double t[BL_NUM] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s <= steps && rc == FDLBM_OK; ++s) {
      for (int k = 0; k < BL_NUM; ++k) {
        if (s > 0) (void)hipEventRecord(ev[2 * k], b->stream);
        const hipError_t e = batch_launch(b, b->cur, 1u << k);
        if (e != hipSuccess) {
          rc = bset_err(b, FDLBM_E_HIP, "autotune launch: %s", hipGetErrorString(e));
          break;
        }
        if (s > 0) (void)hipEventRecord(ev[2 * k + 1], b->stream);
      }
      if (rc != FDLBM_OK) break;
      batch_advance(b, 1);
      if (s > 0) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) {
          rc = bset_err(b, FDLBM_E_HIP, "autotune sync");
          break;
        }
        for (int k = 0; k < BL_NUM; ++k) {
          float ms = 0;
          (void)hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
          t[k] += ms;
        }
      }
    }
    for (int k = 0; k < BL_NUM; ++k)
      if (t[k] < best_t[k]) {
        best_t[k] = t[k];
        best_g[k] = b->grid[k];
      }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < BL_NUM; ++k) b->grid[k] = rc == FDLBM_OK ? best_g[k] : saved[k];
  batch_drop_graphs(b);
  if (grid_out)
    for (int k = 0; k < BL_NUM; ++k) grid_out[k] = b->grid[k];
  return rc;
}
