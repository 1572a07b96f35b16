/*
 * FP64 CPU oracle of the coupled FD-LBM step.  TEST INFRASTRUCTURE ONLY: the
 * product never links or calls this file; it shares no code with it.
 *
 * Written as plain loops that follow the paper's statement of the method in
 * its own order.  Where the paper is silent or garbled, the reading taken is
 * stated at the place it is used (tag "reading:").  The generic machinery here
 * (moment-basis inversion for the source shapes, Lagrange interpolation for the
 * streaming stencils, a dense linear solve for the diffusion-velocity
 * correction) is deliberately different from the closed forms a fast
 * implementation would use, so that agreement between the two is evidence.
 *
 * Every function is pinned by the CPU tests against closed forms,
 * invariants or the paper's printed values.  The one quantity without a
 * reference value is the size of the mass drift of interpolated species
 * next to walls without a reaction (Sec. 4.2 names the error of the
 * one-sided stencils and gives no figure): only its convergence with
 * resolution is pinned.
 */
#include "fdlbm_oracle.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXS ORACLE_MAXS
#define MAXQ 19
#define MAXR ORACLE_MAXR

enum { K_GAS = 0, K_SOLID = 1, K_WALL = 2, K_INLET = 3, K_OUTLET = 4 };

#define F_DIFF 1u
#define F_VISC 2u
#define F_ENER 4u
#define F_PR 8u
/* diagnostic switches for the pin tests (not corrections of their own) */
#define F_NO_QXYZ 16u /* omit the cubic part Q'_xyz of the viscous correction */
#define F_NO_ROFF 32u /* omit the off-diagonal R'_ab of the energy-flux correction */

struct oracle_sim {
  int D, Q;
  int c[MAXQ][3];
  int nx, ny, nz, n;
  int periodic[3];
  int ns;
  int inout;
  int geometry_set, species_set, init_done;
  uint8_t *kind;
  /* species and transport */
  double M[MAXS], cj[MAXS], sj[MAXS], mu0[MAXS], mu_T_exp, Djk0[MAXS * MAXS], D_T_exp,
      D_p_exp, T_ref, p_ref, Pr;
  double Pr_j[MAXS]; /* per-species Prandtl numbers (all Pr unless set separately) */
  /* Lennard-Jones transport (Eq.(26)-(27)): T_unit / eps_j per species and a
   * collision-integral table on a uniform T* grid */
  int lj, lj_n;
  double lj_ie[MAXS], lj_t0, lj_dt, lj_om_mu[64], lj_om_d[64];
  unsigned flags;
  /* solid */
  double alpha_s, C_s, T_bc[6];
  int solid_scheme; /* 0 forward Euler, 1 Crank-Nicolson */
  /* reactions: the rate law of oracle_set_reaction is reaction 0; further
   * ones are appended by oracle_add_reaction */
  int n_rx;
  double rnu[MAXR][MAXS], rorder[MAXR][MAXS], rk0[MAXR], rea[MAXR], rTref[MAXR], rdH[MAXR];
  double T_iso, tol;
  int wall_mode, max_iter;
  /* flow */
  double F[3], X_in[MAXS], p_in, T_in;
  /* source shapes (unscaled, c_j = 1): psi[a], pi[a][b], chi[a], phi */
  double psi[3][MAXQ], pis[3][3][MAXQ], chi[3][MAXQ], phi[MAXQ];
  /* state */
  double *G, *Gn;   /* populations [(j*Q + i)*n + node] */
  double *gpre;     /* streamed (pre-collision) populations, same layout */
  double *Ts, *Tsn;
  /* per-node fields of the current step */
  double *rho, *u, *T, *tau1, *tau2, *Jf, *Uc;
  double *wall_r, *wall_dE;
  double *wall_q;   /* reaction heat per wall node and step, sum_k -dH_k r_k */
  double *acc_node; /* per-node terms of the cumulative sums, added in node order */
  double *wall_u;   /* wall velocity U_w per node, 3 rows (NULL: walls at rest) */
  int literal_eq6;  /* 1: f* at the mixture temperature as printed in Eq.(6) */
  int rate_area;    /* 1: rate scaled by the wall node's wetted area (reading) */
  int src_flux;     /* 1: wall source scaled by 1/c_j (stoichiometric mass flux, reading) */
  int eq48;         /* 1: solid-gas coupling of Eq.(48) instead of the flux-matched one */
  int halfway;      /* 1: wall placed half-way along each link (Sec. 4.3, reading) */
  /* cumulative counters */
  double moles, heat, bheat, work;
  int64_t step;
  char err[256];
};

static int fail(oracle_sim *s, const char *msg) {
  if (s) snprintf(s->err, sizeof s->err, "%s", msg);
  return -1;
}

const char *oracle_error(const oracle_sim *s) { return s ? s->err : "null simulation"; }

/* ------------------------------------------------------------------------ */
/* lattice velocities: Eq.(2) for D2Q9 (rest, +x, +y, -x, -y, diagonals);
 * D3Q19 (reading): rest, +-x, +-y, +-z, then the xy, xz and yz edges.      */
/* ------------------------------------------------------------------------ */
static const int C2[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                             {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
static const int C3[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0},
                              {1, -1, 0}, {1, 0, 1},   {-1, 0, 1}, {-1, 0, -1}, {1, 0, -1},
                              {0, 1, 1},  {0, -1, 1},  {0, -1, -1}, {0, 1, -1}};

static int fill_velocities(int lattice, int c[MAXQ][3]) {
  if (lattice == 2) {
    for (int i = 0; i < 9; ++i) {
      c[i][0] = C2[i][0];
      c[i][1] = C2[i][1];
      c[i][2] = 0;
    }
    return 9;
  }
  if (lattice == 3) {
    for (int i = 0; i < 19; ++i)
      for (int a = 0; a < 3; ++a) c[i][a] = C3[i][a];
    return 19;
  }
  return -1;
}

int oracle_velocities(int lattice, int *c_out) {
  int c[MAXQ][3];
  int Q = fill_velocities(lattice, c);
  if (Q < 0) return -1;
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < 3; ++a) c_out[i * 3 + a] = c[i][a];
  return Q;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium, Eq.(4) and Eq.(6).                                          */
/* ------------------------------------------------------------------------ */
/* One-dimensional factor of Eq.(4) as printed, for lattice component c,
 * scaled velocity U = sqrt(M_j) u and temperature T:
 *   (1 - 2c^2) / 2^(c^2) * [(c^2 - 1) + c U + U^2 + T].
 * Reading: the printed factor is negative for every c (its product of two is
 * positive, so D2Q9 is unaffected); the positive factor is used, i.e. the
 * printed one times -1.  This is required for the 3-D extension. */
static double eq_factor(int c, double U, double T) {
  double c2 = (double)(c * c);
  double printed = (1.0 - 2.0 * c2) / pow(2.0, c2) * ((c2 - 1.0) + c * U + U * U + T);
  return -printed;
}

/* f_i for one species with density rho_j, mass M_j, velocity u, temperature T.
 * D2Q9: the product of Eq.(4) over x and y.
 * D3Q19 (reading; the paper is 2-D only): edge populations (two nonzero
 * components a, b) are rho F_a F_b; face populations (one nonzero component a)
 * are rho F_a (1 - 2T - U_b^2 - U_c^2) with b, c the other axes; the rest
 * population takes the remaining mass.  This reproduces the Maxwellian
 * density, momentum and pressure tensor exactly. */
static void equilibrium(int D, int Q, const int c[MAXQ][3], double rho_j, double M_j,
                        const double *u, double T, double *f) {
  double sq = sqrt(M_j);
  double U[3] = {sq * u[0], sq * u[1], D == 3 ? sq * u[2] : 0.0};
  if (D == 2) {
    for (int i = 0; i < Q; ++i)
      f[i] = rho_j * eq_factor(c[i][0], U[0], T) * eq_factor(c[i][1], U[1], T);
    return;
  }
  double sum = 0.0;
  for (int i = 1; i < Q; ++i) {
    int nzc = 0, axes[3];
    for (int a = 0; a < 3; ++a)
      if (c[i][a] != 0) axes[nzc++] = a;
    if (nzc == 2) {
      f[i] = rho_j * eq_factor(c[i][axes[0]], U[axes[0]], T) *
             eq_factor(c[i][axes[1]], U[axes[1]], T);
    } else {
      int a = axes[0];
      double rest_perp = 1.0 - 2.0 * T;
      for (int b = 0; b < 3; ++b)
        if (b != a) rest_perp -= U[b] * U[b];
      f[i] = rho_j * eq_factor(c[i][a], U[a], T) * rest_perp;
    }
    sum += f[i];
  }
  f[0] = rho_j - sum;
}

int oracle_equilibrium(int lattice, double rho_j, double M_j, const double *u3, double T,
                       double *f_out) {
  int c[MAXQ][3];
  int Q = fill_velocities(lattice, c);
  if (Q < 0) return -1;
  equilibrium(lattice, Q, c, rho_j, M_j, u3, T, f_out);
  return Q;
}

/* ------------------------------------------------------------------------ */
/* Source shapes by moment-basis inversion.                                  */
/* A source with prescribed moments is built as M_B^{-1} applied to the      */
/* moment vector; the basis is the lattice's natural one:                   */
/*  D2Q9  {1, cx, cy, cx^2, cy^2, cxcy, cx c^2, cy c^2, cx^2 cy^2}          */
/*  D3Q19 {1, c_a (3), c_a^2 (3), cxcy, cxcz, cycz, c_a c^2 (3),            */
/*         cx(cy^2-cz^2), cy(cz^2-cx^2), cz(cx^2-cy^2), cx^2cy^2, cy^2cz^2, */
/*         cz^2cx^2}                                                         */
/* With the D2Q9 basis, the unit-x-momentum source is Eq.(13)'s psi_x.      */
/* ------------------------------------------------------------------------ */
static double basis_fn(int D, int k, const int *cv) {
  double x = cv[0], y = cv[1], z = cv[2], c2 = x * x + y * y + z * z;
  if (D == 2) {
    switch (k) {
      case 0: return 1;
      case 1: return x;
      case 2: return y;
      case 3: return x * x;
      case 4: return y * y;
      case 5: return x * y;
      case 6: return x * c2;
      case 7: return y * c2;
      case 8: return x * x * y * y;
    }
    return 0;
  }
  switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x;
    case 5: return y * y;
    case 6: return z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * c2;
    case 11: return y * c2;
    case 12: return z * c2;
    case 13: return x * (y * y - z * z);
    case 14: return y * (z * z - x * x);
    case 15: return z * (x * x - y * y);
    case 16: return x * x * y * y;
    case 17: return y * y * z * z;
    case 18: return z * z * x * x;
  }
  return 0;
}

/* Gauss-Jordan inverse with partial pivoting of an m x m matrix. */
static int invert(int m, double *A, double *Ainv) {
  double W[MAXQ * 2 * MAXQ];
  int w = 2 * m;
  for (int r = 0; r < m; ++r)
    for (int k = 0; k < w; ++k) W[r * w + k] = k < m ? A[r * m + k] : (k - m == r ? 1.0 : 0.0);
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (fabs(W[r * w + col]) > fabs(W[piv * w + col])) piv = r;
    if (fabs(W[piv * w + col]) < 1e-14) return -1;
    if (piv != col)
      for (int k = 0; k < w; ++k) {
        double t = W[col * w + k];
        W[col * w + k] = W[piv * w + k];
        W[piv * w + k] = t;
      }
    double d = W[col * w + col];
    for (int k = 0; k < w; ++k) W[col * w + k] /= d;
    for (int r = 0; r < m; ++r) {
      if (r == col) continue;
      double f = W[r * w + col];
      if (f != 0.0)
        for (int k = 0; k < w; ++k) W[r * w + k] -= f * W[col * w + k];
    }
  }
  for (int r = 0; r < m; ++r)
    for (int k = 0; k < m; ++k) Ainv[r * m + k] = W[r * w + m + k];
  return 0;
}

/* x = A^-1 b for an m x m system (m <= MAXQ) */
static int solve(int m, const double *A, const double *b, double *x) {
  double Ac[MAXQ * MAXQ], Ai[MAXQ * MAXQ];
  memcpy(Ac, A, sizeof(double) * m * m);
  if (invert(m, Ac, Ai)) return -1;
  for (int r = 0; r < m; ++r) {
    x[r] = 0.0;
    for (int k = 0; k < m; ++k) x[r] += Ai[r * m + k] * b[k];
  }
  return 0;
}

/* basis index of each moment a shape prescribes; -1 if absent on the lattice */
static int shape_basis_index(int D, int which) {
  if (D == 2) {
    static const int map2[12] = {1, 2, -1, 3, 4, -1, 5, -1, -1, 6, 7, -1};
    return which < 12 ? map2[which] : -1;
  }
  static const int map3[12] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12};
  return which < 12 ? map3[which] : -1;
}

static int build_shape(int D, int Q, const int c[MAXQ][3], int which, double *out) {
  double B[MAXQ * MAXQ], Binv[MAXQ * MAXQ];
  for (int k = 0; k < Q; ++k)
    for (int i = 0; i < Q; ++i) B[k * Q + i] = basis_fn(D, k, c[i]);
  if (invert(Q, B, Binv)) return -1;
  /* the population vector with unit moment k and zero others is column k of B^-1 */
  if (which == 12) {
    /* energy source: unit energy split equally over the D diagonal second moments */
    for (int i = 0; i < Q; ++i) out[i] = 0.0;
    for (int a = 0; a < D; ++a) {
      int k = shape_basis_index(D, 3 + a);
      for (int i = 0; i < Q; ++i) out[i] += Binv[i * Q + k] / D;
    }
    return 0;
  }
  int k = shape_basis_index(D, which);
  if (k < 0) {
    for (int i = 0; i < Q; ++i) out[i] = 0.0;
    return 1;
  }
  for (int i = 0; i < Q; ++i) out[i] = Binv[i * Q + k];
  return 0;
}

int oracle_shape(int lattice, int which, double *out) {
  int c[MAXQ][3];
  int Q = fill_velocities(lattice, c);
  if (Q < 0 || which < 0 || which > 12) return -1;
  if (build_shape(lattice, Q, c, which, out) < 0) return -1;
  return Q;
}

/* ------------------------------------------------------------------------ */
/* Streaming stencils, Eq.(33)-(36).                                        */
/* Coordinates along the streaming line: a tap at t is node x + (t-1) e_i.  */
/* The value emitted by that node has travelled c_j = 1 - s and sits at      */
/* t - s relative to x, so the pre-collision value at x is the interpolant  */
/* through the taps evaluated at distance s.  The bulk formula Eq.(34) is   */
/* the quadratic through t = -1, 0, 1; Eq.(35) (away from a wall) the one    */
/* through t = 0, 1, 2; Eq.(36) (onto a wall) the one through t = 0, -1, -2.*/
/* Reading for stencils that run out of points (thin throats, concave       */
/* corners): degrade the order (linear through two taps, then one tap).    */
/* ------------------------------------------------------------------------ */
static const int STENCIL_T[7][3] = {{-1, 0, 1}, {0, 1, 2}, {0, -1, -2}, {0, 1, 0},
                                    {-1, 0, 0}, {0, 0, 0},  {1, 0, 0}};
static const int STENCIL_N[7] = {3, 3, 3, 2, 2, 1, 1};

int oracle_interp_weights(int cls, double s, double *w3, int *t3, int *ntaps) {
  if (cls < 0 || cls > 6) return -1;
  int m = STENCIL_N[cls];
  for (int k = 0; k < m; ++k) {
    double L = 1.0;
    for (int q = 0; q < m; ++q)
      if (q != k) L *= (s - STENCIL_T[cls][q]) / (double)(STENCIL_T[cls][k] - STENCIL_T[cls][q]);
    w3[k] = L;
    t3[k] = STENCIL_T[cls][k];
  }
  *ntaps = m;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* geometry helpers                                                          */
/* ------------------------------------------------------------------------ */
static int node_of(const oracle_sim *s, int x, int y, int z) { return x + s->nx * (y + s->ny * z); }

/* node at (node + k*e_i), or -1 outside a non-periodic axis */
static int shift(const oracle_sim *s, int node, int i, int k) {
  int x = node % s->nx, y = (node / s->nx) % s->ny, z = node / (s->nx * s->ny);
  int p[3] = {x + k * s->c[i][0], y + k * s->c[i][1], z + k * s->c[i][2]};
  int lim[3] = {s->nx, s->ny, s->nz};
  for (int a = 0; a < 3; ++a) {
    if (p[a] < 0 || p[a] >= lim[a]) {
      if (!s->periodic[a]) return -1;
      p[a] = ((p[a] % lim[a]) + lim[a]) % lim[a];
    }
  }
  return node_of(s, p[0], p[1], p[2]);
}

/* face neighbour along axis a (dir = +1/-1), -1 if outside */
static int face_nbr(const oracle_sim *s, int node, int a, int dir) {
  int x = node % s->nx, y = (node / s->nx) % s->ny, z = node / (s->nx * s->ny);
  int p[3] = {x, y, z};
  int lim[3] = {s->nx, s->ny, s->nz};
  p[a] += dir;
  if (p[a] < 0 || p[a] >= lim[a]) {
    if (!s->periodic[a]) return -1;
    p[a] = (p[a] + lim[a]) % lim[a];
  }
  return node_of(s, p[0], p[1], p[2]);
}

static int gaslike(const oracle_sim *s, int node) {
  return node >= 0 && (s->kind[node] == K_GAS || s->kind[node] == K_INLET ||
                       s->kind[node] == K_OUTLET);
}

/* Does node y emit a population along direction i?  Gas nodes emit along
 * every direction; a wall node emits its thermalised populations along the
 * directions that point into the gas (the wall sits on the solid node). */
static int emits(const oracle_sim *s, int y, int i) {
  if (y < 0) return 0;
  if (gaslike(s, y)) return 1;
  if (s->kind[y] == K_WALL) return gaslike(s, shift(s, y, i, 1));
  return 0;
}

/* Is (x, i) a streaming destination?  Gas nodes receive along every moving
 * direction; a wall node receives the populations arriving from the gas. */
static int is_destination(const oracle_sim *s, int x, int i) {
  if (i == 0) return 0;
  if (gaslike(s, x)) return 1;
  if (s->kind[x] == K_WALL) return gaslike(s, shift(s, x, i, -1));
  return 0;
}

/* first stencil (in the order central, forward, backward, two-point,
 * one-point) whose taps all emit along i */
static int choose_stencil(const oracle_sim *s, int x, int i) {
  for (int cls = 0; cls < 7; ++cls) {
    int ok = 1;
    for (int k = 0; k < STENCIL_N[cls] && ok; ++k)
      ok = emits(s, shift(s, x, i, STENCIL_T[cls][k] - 1), i);
    if (ok) return cls;
  }
  return -1;
}

static double *pop(oracle_sim *s, double *A, int j, int i, int node) {
  return &A[((size_t)j * s->Q + i) * s->n + node];
}

static double stream_one(oracle_sim *s, int x, int j, int i) {
  int cls = choose_stencil(s, x, i);
  double w[3];
  int t[3], m;
  oracle_interp_weights(cls, s->sj[j], w, t, &m);
  double v = 0.0;
  for (int k = 0; k < m; ++k) v += w[k] * *pop(s, s->G, j, i, shift(s, x, i, t[k] - 1));
  return v;
}

/* ------------------------------------------------------------------------ */
/* creation and parameters                                                   */
/* ------------------------------------------------------------------------ */
oracle_sim *oracle_create(int lattice, int nx, int ny, int nz, const int *periodic,
                          int n_species) {
  if ((lattice != 2 && lattice != 3) || nx < 1 || ny < 1 || nz < 1 || n_species < 1 ||
      n_species > MAXS)
    return NULL;
  if (lattice == 2 && nz != 1) return NULL;
  oracle_sim *s = (oracle_sim *)calloc(1, sizeof(oracle_sim));
  s->D = lattice;
  s->Q = fill_velocities(lattice, s->c);
  s->nx = nx;
  s->ny = ny;
  s->nz = nz;
  s->n = nx * ny * nz;
  for (int a = 0; a < 3; ++a) s->periodic[a] = periodic ? periodic[a] != 0 : 1;
  if (lattice == 2) s->periodic[2] = 1;
  s->ns = n_species;
  size_t np = (size_t)n_species * s->Q * s->n;
  s->G = (double *)calloc(np, sizeof(double));
  s->Gn = (double *)calloc(np, sizeof(double));
  s->gpre = (double *)calloc(np, sizeof(double));
  s->Ts = (double *)calloc(s->n, sizeof(double));
  s->Tsn = (double *)calloc(s->n, sizeof(double));
  s->rho = (double *)calloc((size_t)n_species * s->n, sizeof(double));
  s->u = (double *)calloc((size_t)3 * s->n, sizeof(double));
  s->T = (double *)calloc(s->n, sizeof(double));
  s->tau1 = (double *)calloc((size_t)n_species * s->n, sizeof(double));
  s->tau2 = (double *)calloc((size_t)n_species * s->n, sizeof(double));
  s->Jf = (double *)calloc((size_t)n_species * 3 * s->n, sizeof(double));
  s->Uc = (double *)calloc((size_t)3 * s->n, sizeof(double));
  s->wall_r = (double *)calloc(s->n, sizeof(double));
  s->wall_q = (double *)calloc(s->n, sizeof(double));
  s->wall_dE = (double *)calloc(s->n, sizeof(double));
  s->acc_node = (double *)calloc(s->n, sizeof(double));
  s->kind = (uint8_t *)calloc(s->n, 1);
  if (!s->G || !s->Gn || !s->gpre || !s->Ts || !s->Tsn || !s->rho || !s->u || !s->T ||
      !s->tau1 || !s->tau2 || !s->Jf || !s->Uc || !s->wall_r || !s->wall_dE || !s->wall_q || !s->kind) {
    oracle_destroy(s);
    return NULL;
  }
  for (int w = 0; w < 13; ++w) {
    double tmp[MAXQ];
    build_shape(s->D, s->Q, s->c, w, tmp);
    if (w < 3) memcpy(s->psi[w], tmp, sizeof tmp);
    else if (w < 6) memcpy(s->pis[w - 3][w - 3], tmp, sizeof tmp);
    else if (w < 9) {
      static const int ab[3][2] = {{0, 1}, {0, 2}, {1, 2}};
      memcpy(s->pis[ab[w - 6][0]][ab[w - 6][1]], tmp, sizeof tmp);
    } else if (w < 12) memcpy(s->chi[w - 9], tmp, sizeof tmp);
    else memcpy(s->phi, tmp, sizeof tmp);
  }
  for (int a = 0; a < 6; ++a) s->T_bc[a] = NAN;
  s->Pr = 1.0;
  s->tol = 1e-13;
  s->max_iter = 64;
  return s;
}

void oracle_destroy(oracle_sim *s) {
  if (!s) return;
  free(s->G);
  free(s->Gn);
  free(s->gpre);
  free(s->Ts);
  free(s->Tsn);
  free(s->rho);
  free(s->u);
  free(s->T);
  free(s->tau1);
  free(s->tau2);
  free(s->Jf);
  free(s->Uc);
  free(s->wall_r);
  free(s->wall_q);
  free(s->wall_u);
  free(s->acc_node);
  free(s->wall_dE);
  free(s->kind);
  free(s);
}

int oracle_set_geometry(oracle_sim *s, const uint8_t *mask, int inout) {
  if (!s || !mask) return fail(s, "null argument");
  s->inout = inout;
  if (inout && (s->periodic[0] || s->nx < 6)) return fail(s, "inlet/outlet needs a non-periodic x axis of >= 6 nodes");
  for (int node = 0; node < s->n; ++node) {
    int x = node % s->nx;
    if (mask[node] > 1) return fail(s, "mask values must be 0 (gas) or 1 (solid)");
    if (mask[node] == 0) {
      s->kind[node] = K_GAS;
      if (inout && x <= 1) s->kind[node] = K_INLET;
      if (inout && x >= s->nx - 2) s->kind[node] = K_OUTLET;
    } else {
      if (inout && (x <= 1 || x >= s->nx - 2)) return fail(s, "inlet/outlet planes must be gas");
      s->kind[node] = K_SOLID;
    }
  }
  /* the outlet takes the state of the last interior plane: it must be gas */
  for (int node = 0; node < s->n; ++node)
    if (s->kind[node] == K_OUTLET && s->kind[node - node % s->nx + s->nx - 3] != K_GAS)
      return fail(s, "an outlet row has no gas node at x = nx - 3");
  int n_gas = 0;
  for (int node = 0; node < s->n; ++node) {
    if (gaslike(s, node)) {
      ++n_gas;
      /* a plain gas node must not sit on a closed (non-periodic) domain face */
      if (s->kind[node] == K_GAS)
        for (int i = 1; i < s->Q; ++i)
          if (shift(s, node, i, 1) < 0) return fail(s, "gas touches a non-periodic domain edge");
      continue;
    }
    /* wall node = solid node with at least one gas node among its lattice neighbours */
    for (int i = 1; i < s->Q; ++i)
      if (gaslike(s, shift(s, node, i, 1))) {
        s->kind[node] = K_WALL;
        break;
      }
  }
  if (n_gas == 0) return fail(s, "no gas node");
  s->geometry_set = 1;
  return 0;
}

int oracle_set_species(oracle_sim *s, const double *M, const double *mu0, double mu_T_exp,
                       const double *Djk0, double D_T_exp, double D_p_exp, double T_ref,
                       double p_ref, double Pr, unsigned flags) {
  if (!s || !M || !mu0 || !Djk0) return fail(s, "null argument");
  for (int j = 0; j < s->ns; ++j) {
    if (!(M[j] >= 1.0)) return fail(s, "masses are relative to the lightest species (>= 1)");
    if (!(mu0[j] > 0.0)) return fail(s, "viscosity must be positive");
    s->M[j] = M[j];
    s->cj[j] = sqrt(1.0 / M[j]); /* Eq.(2): c_j = sqrt(M_0 / M_j) */
    s->sj[j] = 1.0 - s->cj[j];   /* off-lattice shift of Eq.(33) */
    s->mu0[j] = mu0[j];
    for (int k = 0; k < s->ns; ++k) {
      s->Djk0[j * MAXS + k] = Djk0[j * s->ns + k];
      if (j != k && !(Djk0[j * s->ns + k] > 0.0)) return fail(s, "binary diffusivities must be positive");
    }
  }
  if (!(T_ref > 0 && p_ref > 0 && Pr > 0)) return fail(s, "T_ref, p_ref, Pr must be positive");
  s->mu_T_exp = mu_T_exp;
  s->D_T_exp = D_T_exp;
  s->D_p_exp = D_p_exp;
  s->T_ref = T_ref;
  s->p_ref = p_ref;
  s->Pr = Pr;
  for (int j = 0; j < MAXS; ++j) s->Pr_j[j] = Pr;
  s->flags = flags;
  s->species_set = 1;
  return 0;
}

/* Per-species Prandtl numbers (Sec. 3, the extension noted after Eq.(21));
 * NULL restores the common value of oracle_set_species. */
int oracle_set_prandtl(oracle_sim *s, const double *Pr_j) {
  if (!s) return fail(s, "null argument");
  for (int j = 0; j < s->ns; ++j) {
    const double v = Pr_j ? Pr_j[j] : s->Pr;
    if (!(v > 0)) return fail(s, "Prandtl numbers must be positive");
  }
  for (int j = 0; j < s->ns; ++j) s->Pr_j[j] = Pr_j ? Pr_j[j] : s->Pr;
  return 0;
}

/* Lennard-Jones transport (Eq.(26)-(27), with the collision integrals from a
 * table on a uniform grid of reduced temperature T* = T T_unit / eps):
 * eps_over_k per species (K), T_unit (K per lattice temperature unit),
 * n >= 2 values of Omega_mu and Omega_D at T* = tmin .. tmax.  eps_over_k
 * NULL: power laws again. */
int oracle_set_lj(oracle_sim *s, const double *eps_over_k, double T_unit, double tmin, double tmax, int n,
                  const double *om_mu, const double *om_d) {
  if (!s) return fail(s, "null argument");
  if (!eps_over_k) {
    s->lj = 0;
    return 0;
  }
  if (!om_mu || !om_d || n < 2 || n > 64 || !(tmax > tmin) || !(tmin > 0) || !(T_unit > 0))
    return fail(s, "bad collision-integral table");
  for (int i = 0; i < n; ++i)
    if (!(om_mu[i] > 0 && om_d[i] > 0)) return fail(s, "collision integrals must be positive");
  for (int j = 0; j < s->ns; ++j) {
    if (!(eps_over_k[j] > 0)) return fail(s, "eps/k must be positive");
    s->lj_ie[j] = T_unit / eps_over_k[j];
  }
  s->lj_n = n;
  s->lj_t0 = tmin;
  s->lj_dt = (tmax - tmin) / (n - 1);
  for (int i = 0; i < n; ++i) {
    s->lj_om_mu[i] = om_mu[i];
    s->lj_om_d[i] = om_d[i];
  }
  s->lj = 1;
  return 0;
}

int oracle_set_solid(oracle_sim *s, double alpha_s, double C_s, const double *T_bc6) {
  if (!s) return fail(s, "null argument");
  /* Eq.(46)-(47): forward Euler is stable only for alpha_s <= 1/(2D); the
   * Crank-Nicolson scheme for any alpha_s */
  if (!(alpha_s >= 0.0)) return fail(s, "alpha_s must be non-negative");
  if (s->solid_scheme == 0 && alpha_s > 0.5 / s->D) return fail(s, "alpha_s out of the stable range");
  if (!(C_s > 0.0)) return fail(s, "C_s must be positive");
  s->alpha_s = alpha_s;
  s->C_s = C_s;
  for (int a = 0; a < 6; ++a) s->T_bc[a] = T_bc6 ? T_bc6[a] : NAN;
  return 0;
}

/* Time scheme of the solid heat equation (Sec. 5: Crank-Nicolson is the
 * recommended extension for alpha_s > 1/(2D)): 0 forward Euler, 1 CN. */
int oracle_set_solid_scheme(oracle_sim *s, int scheme) {
  if (!s) return fail(s, "null argument");
  if (scheme != 0 && scheme != 1) return fail(s, "scheme must be 0 or 1");
  if (scheme == 0 && s->alpha_s > 0.5 / s->D) return fail(s, "alpha_s out of the stable range");
  s->solid_scheme = scheme;
  return 0;
}

/* reaction k's stoichiometry, orders and rate constants */
static int put_reaction(oracle_sim *s, int k, const double *nu, const double *order, double k0,
                        double ea, double T_ref, double dH) {
  for (int j = 0; j < s->ns; ++j)
    if (order[j] < 0) return fail(s, "negative reaction order");
  for (int j = 0; j < s->ns; ++j) {
    s->rnu[k][j] = nu[j];
    s->rorder[k][j] = order[j];
  }
  s->rk0[k] = k0;
  s->rea[k] = ea;
  s->rTref[k] = T_ref;
  s->rdH[k] = dH;
  return 0;
}

int oracle_set_reaction(oracle_sim *s, const double *nu, const double *order, double k0,
                        double ea, double T_ref, double dH, int wall_mode, double T_iso,
                        double tol, int max_iter) {
  if (!s || !nu || !order) return fail(s, "null argument");
  if (put_reaction(s, 0, nu, order, k0, ea, T_ref, dH)) return -1;
  s->n_rx = 1;
  s->wall_mode = wall_mode;
  s->T_iso = T_iso;
  s->tol = tol;
  s->max_iter = max_iter;
  return 0;
}

/* a further surface reaction at every wall node (the paper's flux boundary
 * condition takes any source S_j; with several reactions S_j is the sum of
 * their contributions, reading) */
int oracle_add_reaction(oracle_sim *s, const double *nu, const double *order, double k0, double ea,
                        double T_ref, double dH) {
  if (!s || !nu || !order) return fail(s, "null argument");
  if (s->n_rx < 1) return fail(s, "set the first reaction with oracle_set_reaction");
  if (s->n_rx >= MAXR) return fail(s, "too many reactions");
  if (put_reaction(s, s->n_rx, nu, order, k0, ea, T_ref, dH)) return -1;
  s->n_rx++;
  return 0;
}

int oracle_set_flow(oracle_sim *s, const double *F3, const double *X_in, double p_in,
                    double T_in) {
  if (!s) return fail(s, "null argument");
  for (int a = 0; a < 3; ++a) s->F[a] = F3 ? F3[a] : 0.0;
  if (s->D == 2) s->F[2] = 0.0;
  for (int j = 0; j < s->ns; ++j) s->X_in[j] = X_in ? X_in[j] : 0.0;
  s->p_in = p_in;
  s->T_in = T_in;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* transport, Eq.(7)-(8), (14)-(17)                                          */
/* ------------------------------------------------------------------------ */
/* collision integral at reduced temperature ts from the table: linear
 * interpolation on the uniform grid, constant beyond its ends */
static double lj_omega(const oracle_sim *s, const double *om, double ts) {
  double f = (ts - s->lj_t0) / s->lj_dt;
  if (f <= 0.0) return om[0];
  if (f >= s->lj_n - 1) return om[s->lj_n - 1];
  int i = (int)f;
  double w = f - i;
  return (1.0 - w) * om[i] + w * om[i + 1];
}

static void transport(const oracle_sim *s, const double *rho, double T, double *tau1,
                      double *tau2) {
  int ns = s->ns;
  double Cj[MAXS], C = 0.0, Xh[MAXS], Yh[MAXS], sX = 0.0, sMX = 0.0;
  for (int j = 0; j < ns; ++j) {
    Cj[j] = rho[j] / s->M[j];
    C += Cj[j];
  }
  /* reading: the mixing rules use mole fractions floored at 1e-6 and
   * renormalised, so absent species do not divide by zero */
  for (int j = 0; j < ns; ++j) {
    Xh[j] = fmax(Cj[j] / C, 1e-6);
    sX += Xh[j];
  }
  for (int j = 0; j < ns; ++j) {
    Xh[j] /= sX;
    sMX += s->M[j] * Xh[j];
  }
  for (int j = 0; j < ns; ++j) Yh[j] = s->M[j] * Xh[j] / sMX;
  /* species viscosities: power laws, or with Lennard-Jones collision
   * integrals (Eq.(26): mu_j ~ sqrt(M_j T) / (sigma_j^2 Omega_mu(T*_j))),
   * scaled from the reference value mu0_j at T_ref so that sigma_j and the
   * unit constants drop out */
  double mu[MAXS];
  for (int j = 0; j < ns; ++j) {
    if (s->lj)
      mu[j] = s->mu0[j] * sqrt(T / s->T_ref) * lj_omega(s, s->lj_om_mu, s->T_ref * s->lj_ie[j]) /
              lj_omega(s, s->lj_om_mu, T * s->lj_ie[j]);
    else
      mu[j] = s->mu0[j] * pow(T / s->T_ref, s->mu_T_exp);
  }
  /* Wilke, Eq.(15) with the square of the bracket restored (phi_jj = 1) */
  for (int j = 0; j < ns; ++j) {
    double den = 0.0;
    for (int k = 0; k < ns; ++k) {
      double br = 1.0 + sqrt(mu[j] / mu[k]) * pow(s->M[k] / s->M[j], 0.25);
      double phi = br * br / (sqrt(8.0) * sqrt(1.0 + s->M[j] / s->M[k]));
      den += Xh[k] * phi;
    }
    tau1[j] = mu[j] / (C * T * den); /* Eq.(17) */
  }
  if (ns == 1) {
    tau2[0] = tau1[0]; /* f* = f^eq for one species: tau2 never acts */
    return;
  }
  double p = C * T;
  for (int j = 0; j < ns; ++j) {
    double sum = 0.0;
    for (int k = 0; k < ns; ++k) {
      if (k == j) continue;
      double Djk;
      if (s->lj) {
        /* Eq.(27) with T^(3/2) and 1/p; eps_jk = sqrt(eps_j eps_k) */
        double ie = sqrt(s->lj_ie[j] * s->lj_ie[k]);
        Djk = s->Djk0[j * MAXS + k] * pow(T / s->T_ref, 1.5) * (s->p_ref / p) *
              lj_omega(s, s->lj_om_d, s->T_ref * ie) / lj_omega(s, s->lj_om_d, T * ie);
      } else {
        Djk = s->Djk0[j * MAXS + k] * pow(T / s->T_ref, s->D_T_exp) * pow(s->p_ref / p, s->D_p_exp);
      }
      sum += Xh[k] / Djk;
    }
    double Dj = (1.0 - Yh[j]) / sum; /* Eq.(8) */
    /* Eq.(7): tau2 = rho_j D_j / (X_j p); rho_j / (X_j p) = M_j / T exactly */
    tau2[j] = s->M[j] * Dj / T;
  }
}

int oracle_transport(oracle_sim *s, const double *rho, double T, double *tau1, double *tau2) {
  if (!s || !s->species_set) return fail(s, "species not set");
  transport(s, rho, T, tau1, tau2);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* initial state                                                             */
/* ------------------------------------------------------------------------ */
/* Eq.(39): the wall's thermalised populations per unit density,
 * f^eq_ji(1, U_w, T_w) of species j (species independent at U_w = 0) */
static double wall_weight(const oracle_sim *s, int w, int j, int i, double Tw) {
  double f[MAXQ], uw[3] = {0, 0, 0};
  if (s->wall_u)
    for (int a = 0; a < 3; ++a) uw[a] = s->wall_u[(size_t)a * s->n + w];
  equilibrium(s->D, s->Q, s->c, 1.0, s->M[j], uw, Tw, f);
  return f[i];
}

/* velocity of the wall at node w (Eq.(39)'s U_w; zero unless set) */
int oracle_set_wall_velocity(oracle_sim *s, const double *u3) {
  if (!s) return fail(s, "null simulation");
  free(s->wall_u);
  s->wall_u = NULL;
  if (!u3) return 0;
  s->wall_u = (double *)malloc(sizeof(double) * 3 * (size_t)s->n);
  memcpy(s->wall_u, u3, sizeof(double) * 3 * (size_t)s->n);
  return 0;
}

static double wall_temperature(const oracle_sim *s, int w) {
  return s->wall_mode == 1 ? s->T_iso : s->Ts[w];
}

/* Emission weight of the wall node w along link i (into the gas node
 * x = w + e_i) for species j, per unit wall density.
 * Default: the wall sits on the solid node and thermalises at its own state,
 * f^eq_ji(1, U_w, T_w) (Eq.(39)).
 * Option (reading of Sec. 4.3's half-way wall, whose interpolation step the
 * paper leaves to the work it cites): the wall sits half-way along each link.
 * The state the wall node emits at is the one that puts the wall's values at
 * the link's midpoint when interpolated linearly with the gas node x: velocity
 * 2 U_w - u(x) and temperature 2 T_w - T(x), with u(x) and T(x) from x's
 * latest moments (the previous step).  The wall density still solves the
 * mass balance of Eq.(41) with these weights, so mass and (through Delta
 * E_gas) energy stay conserved link by link. */
static double emit_weight(const oracle_sim *s, int w, int j, int i, double Tw) {
  if (!s->halfway) return wall_weight(s, w, j, i, Tw);
  size_t n = (size_t)s->n;
  int x = shift(s, w, i, 1);
  double ul[3], f[MAXQ];
  for (int a = 0; a < 3; ++a) {
    double uw = s->wall_u ? s->wall_u[(size_t)a * n + w] : 0.0;
    ul[a] = 2.0 * uw - s->u[(size_t)a * n + x];
  }
  if (s->D == 2) ul[2] = 0.0;
  equilibrium(s->D, s->Q, s->c, 1.0, s->M[j], ul, 2.0 * Tw - s->T[x], f);
  return f[i];
}

/* reading: initial populations g = f^eq of the given state; wall nodes emit
 * rho_w w_i(T_w) with rho_w the mean of the given densities of their gas
 * link partners */
int oracle_init_fields(oracle_sim *s, const double *rho, const double *u, const double *T,
                       const double *Ts) {
  if (!s || !s->geometry_set || !s->species_set) return fail(s, "geometry/species not set");
  if (!rho || !u || !T || !Ts) return fail(s, "null argument");
  int n = s->n, Q = s->Q;
  memset(s->G, 0, sizeof(double) * (size_t)s->ns * Q * n);
  for (int node = 0; node < n; ++node) {
    s->Ts[node] = Ts[node];
    if (!gaslike(s, node)) continue;
    for (int j = 0; j < s->ns; ++j) {
      double f[MAXQ], uu[3] = {u[node], u[n + node], u[2 * n + node]};
      if (s->D == 2) uu[2] = 0.0;
      equilibrium(s->D, Q, s->c, rho[(size_t)j * n + node], s->M[j], uu, T[node], f);
      for (int i = 0; i < Q; ++i) *pop(s, s->G, j, i, node) = f[i];
      s->rho[(size_t)j * n + node] = rho[(size_t)j * n + node];
    }
    /* the gas state before the first step (read by the half-way wall) */
    for (int a = 0; a < 3; ++a) s->u[(size_t)a * n + node] = a < s->D ? u[(size_t)a * n + node] : 0.0;
    s->T[node] = T[node];
  }
  for (int node = 0; node < n; ++node) {
    if (s->kind[node] != K_WALL) continue;
    double Tw = wall_temperature(s, node);
    for (int j = 0; j < s->ns; ++j) {
      double sum = 0.0;
      int cnt = 0;
      for (int i = 1; i < Q; ++i) {
        int y = shift(s, node, i, 1);
        if (gaslike(s, y)) {
          sum += rho[(size_t)j * n + y];
          ++cnt;
        }
      }
      double rw = sum / cnt;
      for (int i = 1; i < Q; ++i)
        if (gaslike(s, shift(s, node, i, 1))) *pop(s, s->G, j, i, node) = rw * wall_weight(s, node, j, i, Tw);
    }
  }
  s->moles = s->heat = s->bheat = s->work = 0.0;
  s->step = 0;
  s->init_done = 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* the step                                                                  */
/* ------------------------------------------------------------------------ */

/* 1. streaming into every destination, Eq.(33)-(36) */
static void stream_all(oracle_sim *s) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < s->n; ++x) {
    if (gaslike(s, x))
      for (int j = 0; j < s->ns; ++j) *pop(s, s->gpre, j, 0, x) = *pop(s, s->G, j, 0, x);
    for (int i = 1; i < s->Q; ++i) {
      if (!is_destination(s, x, i)) continue;
      for (int j = 0; j < s->ns; ++j) *pop(s, s->gpre, j, i, x) = stream_one(s, x, j, i);
    }
  }
}

/* rate law of reaction k, Eq.(50) generalised: r = k(T_w) prod_m C_m^order_m
 * with the Arrhenius factor k = k0 exp[ea (1 - T_ref / T_w)]
 * (ea = E_a / (R T_ref)) */
static double rate(const oracle_sim *s, int k, const double *rhow, double Tw) {
  double r = s->rk0[k] * exp(s->rea[k] * (1.0 - s->rTref[k] / Tw));
  for (int m = 0; m < s->ns; ++m)
    if (s->rorder[k][m] != 0.0) r *= pow(rhow[m] / s->M[m], s->rorder[k][m]);
  return r;
}

/* 2. reactive diffusive wall, Eq.(37)-(41), P:wall-on-solid-node, Eq.(42) */
static void wall_bc(oracle_sim *s) {
  int Q = s->Q, ns = s->ns;
#pragma omp parallel for schedule(static)
  for (int w = 0; w < s->n; ++w) {
    if (s->kind[w] != K_WALL) continue;
    double Tw = wall_temperature(s, w);
    /* reading (link counting): the populations leaving the gas towards the
     * wall are those on links w - e_i -> w from a gas node (set I_w); the
     * wall emits along every link w -> w + e_i into a gas node (set O_w).
     * For a flat wall the |c.n| weights of Eq.(38)-(39) are all equal to
     * c_j and cancel against the c_j of S_j (Eq.(50)), leaving the per-link
     * lattice mass balance below. */
    double A[MAXS] = {0}, Ein = 0.0, Z[MAXS] = {0};
    for (int i = 1; i < Q; ++i) {
      if (is_destination(s, w, i)) {
        double c2 = (double)(s->c[i][0] * s->c[i][0] + s->c[i][1] * s->c[i][1] +
                             s->c[i][2] * s->c[i][2]);
        for (int j = 0; j < ns; ++j) {
          double g = *pop(s, s->gpre, j, i, w);
          A[j] += g;
          Ein += s->cj[j] * s->cj[j] * c2 * g;
        }
      }
      if (emits(s, w, i))
        for (int j = 0; j < ns; ++j) Z[j] += emit_weight(s, w, j, i, Tw);
    }
    /* Eq.(40)-(41): emitted populations rho_w f^eq(1, U_w, T_w); the wall
     * density of species j satisfies rho_w Z_j = A_j + nu_j M_j r, i.e. the
     * lattice mass of species j grows by nu_j M_j r per wall node and step
     * (the sign reading of S_j: net production into the gas).
     * The paper's fixed-point iteration for rho_w, started here from the
     * non-reactive wall density A_j / Z; each pass treats a reactant's own
     * concentration implicitly (rho_j = A_j / (Z + |nu_j| r / C_j)). */
    /* One reaction term S_j per wall node, also at corners: corner nodes
     * differ from plane ones only in which populations enter Eq.(41)
     * (Sec. 4.3, after the wall-density iteration; the paper builds its
     * walls from plane and convex corner nodes only).  Option (reading, for
     * geometries with concave corners such as sphere packs): the rate is a
     * flux per unit wall area, so it is scaled by the node's wetted area,
     * its rest emission weight over the links into the gas relative to a
     * plane wall's T_w / 2 (factor 1 on plane walls). */
    double area = 1.0;
    if (s->rate_area) {
      double Zg = 0.0, f0[MAXQ], u0[3] = {0, 0, 0};
      equilibrium(s->D, s->Q, s->c, 1.0, 1.0, u0, Tw, f0);
      for (int i = 1; i < Q; ++i)
        if (emits(s, w, i)) Zg += f0[i];
      area = Zg / (0.5 * Tw);
    }
    /* Source in population units per unit of nu_j M_j r: 1 (default: the
     * flux sums of Eq.(38)-(40) taken with the species velocities c_j e_i,
     * so that S_j / c_j = nu_j M_j r is added at the wall), or, as an
     * option, 1 / c_j: the wall adds the population mass that interpolated
     * streaming, which moves a population c_j of a link per step, carries
     * away as the mass flux nu_j M_j r (stoichiometric delivery, the product
     * balance of Sec. 7). */
    double srcf[MAXS];
    for (int j = 0; j < ns; ++j) srcf[j] = s->src_flux ? 1.0 / s->cj[j] : 1.0;
    /* Several reactions (reading): S_j sums the reactions' terms.  The
     * iteration updates the species some reaction consumes with a positive
     * order; each pass treats such a species' own concentration implicitly
     * in the reactions that consume it and takes the reactions that produce
     * it at the current densities.  The other species keep A_j / Z_j until
     * the final balance (they do not enter a rate that consumes them). */
    int upd[MAXS];
    for (int j = 0; j < ns; ++j) {
      upd[j] = 0;
      for (int k = 0; k < s->n_rx; ++k)
        if (s->rnu[k][j] < 0.0 && s->rorder[k][j] > 0.0) upd[j] = 1;
    }
    double rw[MAXS];
    for (int j = 0; j < ns; ++j) rw[j] = A[j] / Z[j];
    for (int it = 0; it < s->max_iter; ++it) {
      double nw[MAXS], rk[MAXR], dmax = 0.0;
      for (int k = 0; k < s->n_rx; ++k) rk[k] = area * rate(s, k, rw, Tw);
      for (int j = 0; j < ns; ++j) {
        nw[j] = rw[j];
        if (upd[j]) {
          double num = 0.0, den = 0.0;
          for (int k = 0; k < s->n_rx; ++k) {
            if (s->rnu[k][j] < 0.0 && s->rorder[k][j] > 0.0) {
              /* r_k / C_j with C_j's own power lowered by one */
              double R = area * s->rk0[k] * exp(s->rea[k] * (1.0 - s->rTref[k] / Tw));
              for (int m = 0; m < ns; ++m) {
                double o = s->rorder[k][m] - (m == j ? 1.0 : 0.0);
                if (o != 0.0) R *= pow(rw[m] / s->M[m], o);
              }
              den += s->rnu[k][j] * srcf[j] * R;
            } else if (s->rnu[k][j] != 0.0) {
              num += s->rnu[k][j] * s->M[j] * srcf[j] * rk[k];
            }
          }
          nw[j] = (A[j] + num) / (Z[j] - den);
        }
        double d = fabs(nw[j] - rw[j]) / fmax(fabs(nw[j]), 1e-300);
        if (d > dmax) dmax = d;
      }
      for (int j = 0; j < ns; ++j) rw[j] = nw[j];
      if (dmax <= s->tol) break;
    }
    /* final rates, and the wall densities from the exact mass balance at them */
    double rk[MAXR], r = 0.0, q = 0.0;
    for (int k = 0; k < s->n_rx; ++k) rk[k] = area * rate(s, k, rw, Tw);
    for (int j = 0; j < ns; ++j) {
      double src = 0.0;
      for (int k = 0; k < s->n_rx; ++k) src += s->rnu[k][j] * s->M[j] * srcf[j] * rk[k];
      rw[j] = (A[j] + src) / Z[j];
    }
    /* total rate (moles reacted per node and step) and reaction heat, Eq.(42) */
    for (int k = 0; k < s->n_rx; ++k) {
      r += rk[k];
      q += -s->rdH[k] * rk[k];
    }
    double Eout = 0.0;
    for (int i = 1; i < Q; ++i) {
      if (!emits(s, w, i)) continue;
      double c2 = (double)(s->c[i][0] * s->c[i][0] + s->c[i][1] * s->c[i][1] +
                           s->c[i][2] * s->c[i][2]);
      for (int j = 0; j < ns; ++j) {
        double W = rw[j] * emit_weight(s, w, j, i, Tw);
        *pop(s, s->Gn, j, i, w) = W;
        Eout += s->cj[j] * s->cj[j] * c2 * W;
      }
    }
    s->wall_r[w] = r;
    s->wall_q[w] = q;
    s->wall_dE[w] = 0.5 * (Eout - Ein); /* kinetic energy handed to the gas */
    /* wall state seen by the gradient stencils of neighbouring gas nodes */
    for (int j = 0; j < ns; ++j) s->rho[(size_t)j * s->n + w] = rw[j];
    for (int a = 0; a < 3; ++a) s->u[(size_t)a * s->n + w] = s->wall_u ? s->wall_u[(size_t)a * s->n + w] : 0.0;
    s->T[w] = Tw;
  }
}

/* 3. moments and transport at gas nodes, Eq.(3), (5), (7)-(8), (11), (14)-(17), (25) */
static void moments(oracle_sim *s) {
  int Q = s->Q, ns = s->ns, n = s->n, D = s->D;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n; ++x) {
    if (!gaslike(s, x)) continue;
    double rho[MAXS], Jg[MAXS][3], E = 0.0, rhot = 0.0, C = 0.0;
    for (int j = 0; j < ns; ++j) {
      rho[j] = 0.0;
      Jg[j][0] = Jg[j][1] = Jg[j][2] = 0.0;
      for (int i = 0; i < Q; ++i) {
        double g = *pop(s, s->gpre, j, i, x);
        rho[j] += g;
        for (int a = 0; a < 3; ++a) Jg[j][a] += s->cj[j] * s->c[i][a] * g;
        double c2 = (double)(s->c[i][0] * s->c[i][0] + s->c[i][1] * s->c[i][1] +
                             s->c[i][2] * s->c[i][2]);
        E += s->cj[j] * s->cj[j] * c2 * g;
      }
      rhot += rho[j];
      C += rho[j] / s->M[j];
    }
    /* mixture velocity of f: the diffusion-velocity correction makes the
     * collision conserve total momentum, so J(f) = J(g) + (1/2) rho F */
    double u[3], u2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double J = 0.0;
      for (int j = 0; j < ns; ++j) J += Jg[j][a];
      u[a] = (J + 0.5 * rhot * s->F[a]) / rhot;
      u2 += u[a] * u[a];
    }
    /* temperature from the energy, Eq.(5) in D dimensions (E = D C T + rho u^2),
     * before the energy of the source terms is added (added in pass 2) */
    double T = (E - rhot * u2) / (D * C);
    double tau1[MAXS], tau2[MAXS];
    transport(s, rho, T, tau1, tau2);
    /* Eq.(25) for each species together with Eq.(11), solved as one linear
     * system per axis for the unknowns J_1(f) .. J_N(f) and U^c:
     *   (1 + a_j) J_j - a_j rho_j U = J_j(g) + a_j rho_j u + rho_j F / 2,
     *   sum_j (J_j - rho_j u) / tau2_j - U sum_j rho_j / tau2_j = 0,
     * with a_j = 1 / (2 tau2_j); the U term in the first line is
     * (1/2) sum_i c Psi^(I) of Eq.(12). */
    for (int a = 0; a < 3; ++a) {
      int m = ns + 1;
      double A[(MAXS + 1) * (MAXS + 1)], b[MAXS + 1];
      memset(A, 0, sizeof A);
      int corr = (s->flags & F_DIFF) && ns > 1;
      for (int j = 0; j < ns; ++j) {
        double aj = 0.5 / tau2[j];
        A[j * m + j] = 1.0 + aj;
        A[j * m + ns] = corr ? -aj * rho[j] : 0.0;
        b[j] = Jg[j][a] + aj * rho[j] * u[a] + 0.5 * rho[j] * s->F[a];
        A[ns * m + j] = corr ? 1.0 / tau2[j] : 0.0;
      }
      double sr = 0.0, sru = 0.0;
      for (int j = 0; j < ns; ++j) {
        sr += rho[j] / tau2[j];
        sru += rho[j] * u[a] / tau2[j];
      }
      A[ns * m + ns] = corr ? -sr : 1.0;
      b[ns] = corr ? sru : 0.0;
      double v[MAXS + 1];
      solve(m, A, b, v);
      for (int r = 0; r < ns; ++r) s->Jf[((size_t)r * 3 + a) * n + x] = v[r];
      s->Uc[(size_t)a * n + x] = v[ns];
    }
    for (int j = 0; j < ns; ++j) {
      s->rho[(size_t)j * n + x] = rho[j];
      s->tau1[(size_t)j * n + x] = tau1[j];
      s->tau2[(size_t)j * n + x] = tau2[j];
    }
    for (int a = 0; a < 3; ++a) s->u[(size_t)a * n + x] = u[a];
    s->T[x] = T;
  }
}

/* values of a face neighbour used by the gradient stencils (reading: central
 * differences over face neighbours; a wall neighbour supplies the wall state
 * rho_w, u = 0, T_w; a missing neighbour at an open domain end repeats x) */
typedef struct {
  double rho[MAXS], u[3], T, tau1[MAXS];
  int is_wall, missing;
} nbstate;

static void get_nb(const oracle_sim *s, int x, int nb, nbstate *o) {
  int n = s->n;
  int y = nb >= 0 && (gaslike(s, nb) || s->kind[nb] == K_WALL) ? nb : x;
  o->missing = nb < 0 || y == x;
  o->is_wall = nb >= 0 && s->kind[nb] == K_WALL;
  for (int j = 0; j < s->ns; ++j) {
    o->rho[j] = s->rho[(size_t)j * n + y];
    o->tau1[j] = o->is_wall ? s->tau1[(size_t)j * n + x] : s->tau1[(size_t)j * n + y];
  }
  for (int a = 0; a < 3; ++a) o->u[a] = s->u[(size_t)a * n + y];
  o->T = s->T[y];
}

/* third-moment deviation of the lattice equilibrium from the Maxwellian
 * (physical units, species j): Q'_aaa and, in 3-D, Q'_xyz */
static double Qdev_aaa(const oracle_sim *s, int j, const nbstate *v, int a) {
  return v->rho[j] / s->M[j] * v->u[a] * (1.0 - 3.0 * v->T) - v->rho[j] * pow(v->u[a], 3);
}
static double Qdev_xyz(int j, const nbstate *v) { return -v->rho[j] * v->u[0] * v->u[1] * v->u[2]; }

/* energy-flux deviation R'_ab = R^lattice - R^Maxwell (physical units) */
static double Rdev(const oracle_sim *s, int j, const nbstate *v, int a, int b) {
  double M = s->M[j], T = v->T, r = v->rho[j];
  double u2 = v->u[0] * v->u[0] + v->u[1] * v->u[1] + v->u[2] * v->u[2];
  if (a == b)
    return r * (T * (1.0 - 3.0 * T) / (M * M) + v->u[a] * v->u[a] * (1.0 - 6.0 * T) / M -
                pow(v->u[a], 4));
  return r * v->u[a] * v->u[b] * ((2.0 - (s->D + 4.0) * T) / M - u2);
}

/* 4-5. sources, temperature of f, equilibria and the collision, Eq.(24) */
static void collide(oracle_sim *s) {
  int Q = s->Q, ns = s->ns, n = s->n, D = s->D;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n; ++x) {
    s->acc_node[x] = 0.0;
    if (!gaslike(s, x)) continue;
    nbstate me, nbp[3], nbm[3];
    get_nb(s, x, x, &me);
    me.missing = 0;
    me.is_wall = 0;
    for (int a = 0; a < D; ++a) {
      get_nb(s, x, face_nbr(s, x, a, +1), &nbp[a]);
      get_nb(s, x, face_nbr(s, x, a, -1), &nbm[a]);
    }
    double C = 0.0, rhot = 0.0;
    for (int j = 0; j < ns; ++j) {
      C += me.rho[j] / s->M[j];
      rhot += me.rho[j];
    }
    /* work of the body force this step, rho u.F (half the trace of its source) */
    s->acc_node[x] = rhot * (me.u[0] * s->F[0] + me.u[1] * s->F[1] + me.u[2] * s->F[2]);
    double S[MAXS][MAXQ];
    double esum = 0.0;
    for (int j = 0; j < ns; ++j) {
      double m[3] = {0, 0, 0}, P[3][3] = {{0}}, Y[3] = {0, 0, 0}, e = 0.0;
      double tau2 = s->tau2[(size_t)j * n + x];
      for (int a = 0; a < D; ++a) {
        /* Eq.(12): Psi^(I) carries momentum rho_j U^c / tau2_j */
        if ((s->flags & F_DIFF) && ns > 1) m[a] += me.rho[j] * s->Uc[(size_t)a * n + x] / tau2;
        /* reading: body force as a source with momentum rho_j F and second
         * moment rho_j (u F + F u) (its trace is the work of the force) */
        m[a] += me.rho[j] * s->F[a];
        for (int b = 0; b < D; ++b) P[a][b] += me.rho[j] * (me.u[a] * s->F[b] + me.u[b] * s->F[a]);
      }
      if (s->flags & F_VISC) {
        /* reading: viscous correction with second moments d_c Q'_abc */
        /* reading at walls: no correction flux crosses a gas-wall face, i.e. a
         * wall neighbour contributes the mirrored value -Q'(x) (the face average
         * vanishes), so the energy this source carries stays in the gas */
        for (int a = 0; a < D; ++a) {
          double qx = Qdev_aaa(s, j, &me, a);
          double qp = nbp[a].is_wall ? -qx : Qdev_aaa(s, j, &nbp[a], a);
          double qm = nbm[a].is_wall ? -qx : Qdev_aaa(s, j, &nbm[a], a);
          P[a][a] += 0.5 * (qp - qm);
        }
        if (D == 3 && !(s->flags & F_NO_QXYZ)) {
          P[0][1] += 0.5 * (Qdev_xyz(j, &nbp[2]) - Qdev_xyz(j, &nbm[2]));
          P[0][2] += 0.5 * (Qdev_xyz(j, &nbp[1]) - Qdev_xyz(j, &nbm[1]));
          P[1][2] += 0.5 * (Qdev_xyz(j, &nbp[0]) - Qdev_xyz(j, &nbm[0]));
          P[1][0] = P[0][1];
          P[2][0] = P[0][2];
          P[2][1] = P[1][2];
        }
      }
      if (s->flags & F_ENER) {
        /* reading: the energy-flux correction removes the deviation R'_ab of
         * the lattice's energy flux (c_a c_b c^2 moment) from the
         * Maxwellian's.  Off-diagonal part: a source with moments
         * sum_i c_a c^2 S = d_b R'_ab (b != a), which the streaming turns
         * into a heat-flux correction.  Diagonal part (at rest the
         * heat-conduction defect, R'_aa = rho T (1 - 3T) / M^2): carried as
         * the divergence of that heat flux, -tau1 d_a R'_aa, in the compact
         * face-flux form of the Prandtl term -- an energy source
         * e = sum over faces of (-tau1 face average) (R'_aa(nb) - R'_aa(x)),
         * no flux through gas-wall faces.  A source's energy moment counts in
         * full in the trapezoidal step, which fixes the factor tau1.  (The
         * same term as a flux moment, d_a R'_aa, makes the step linearly
         * unstable: D2Q9 at every tau1, D3Q19 with a mean flow at small
         * tau1.) */
        for (int a = 0; a < D; ++a)
          for (int b = 0; b < D; ++b)
            if (b != a && !(s->flags & F_NO_ROFF))
              Y[a] += 0.5 * (Rdev(s, j, &nbp[b], a, b) - Rdev(s, j, &nbm[b], a, b));
        const double tx = s->tau1[(size_t)j * n + x];
        for (int a = 0; a < D; ++a) {
          const double rx = Rdev(s, j, &me, a, a);
          const nbstate *nb[2] = {&nbp[a], &nbm[a]};
          for (int q = 0; q < 2; ++q) {
            if (nb[q]->is_wall || nb[q]->missing) continue;
            e += -0.5 * (tx + nb[q]->tau1[j]) * (Rdev(s, j, nb[q], a, a) - rx);
          }
        }
      }
      if ((s->flags & F_PR) && s->Pr_j[j] != 1.0) {
        /* Eq.(19)-(21): Phi^Pr = phi_ji d_a q^Pr_ja with, reading, the species
         * heat capacity c_p,j = (D+2)/(2 M_j), so
         * q^Pr_j = (D+2)(1/Pr_j - 1) tau1_j C_j T dT / M_j (zero at Pr_j = 1;
         * Pr_j = Pr for every species unless set per species, the extension
         * Sec. 3 mentions after Eq.(21)); compact face-flux form with
         * arithmetic face averages; wall faces carry no correction flux
         * (gas-solid exchange is the kinetic wall's). */
        const double kprj = (D + 2.0) * (1.0 / s->Pr_j[j] - 1.0);
        double Kx = kprj * s->tau1[(size_t)j * n + x] * me.rho[j] / s->M[j] * me.T / s->M[j];
        for (int a = 0; a < D; ++a) {
          const nbstate *nb[2] = {&nbp[a], &nbm[a]};
          for (int q = 0; q < 2; ++q) {
            if (nb[q]->is_wall || nb[q]->missing) continue;
            double Kn = kprj * nb[q]->tau1[j] * nb[q]->rho[j] / s->M[j] * nb[q]->T / s->M[j];
            e += 0.5 * (Kx + Kn) * (nb[q]->T - me.T);
          }
        }
      }
      /* population-space source: shapes scaled to species velocities c_j c_0i */
      double cjv = s->cj[j];
      for (int i = 0; i < Q; ++i) {
        double v = 0.0;
        for (int a = 0; a < D; ++a) {
          v += s->psi[a][i] * m[a] / cjv;
          v += s->pis[a][a][i] * P[a][a] / (cjv * cjv);
          v += s->chi[a][i] * Y[a] / (cjv * cjv * cjv);
          for (int b = a + 1; b < D; ++b) v += s->pis[a][b][i] * P[a][b] / (cjv * cjv);
        }
        v += s->phi[i] * e / (cjv * cjv);
        S[j][i] = v;
        double c2 = (double)(s->c[i][0] * s->c[i][0] + s->c[i][1] * s->c[i][1] +
                             s->c[i][2] * s->c[i][2]);
        esum += cjv * cjv * c2 * v;
      }
    }
    /* Eq.(25), third line, generalised: T(f) adds half the source energy */
    double Tf = me.T + esum / (2.0 * D * C);
    /* species velocities u_j = J_j(f) / rho_j */
    double uj[MAXS][3], ediff = 0.0;
    for (int j = 0; j < ns; ++j)
      for (int a = 0; a < 3; ++a) {
        uj[j][a] = me.rho[j] > 1e-300 ? s->Jf[((size_t)j * 3 + a) * n + x] / me.rho[j] : me.u[a];
        ediff += me.rho[j] * (uj[j][a] - me.u[a]) * (uj[j][a] - me.u[a]);
      }
    /* Reading for Eq.(6): the auxiliary state is the quasi-equilibrium with the
     * species densities and momenta and the mixture energy held fixed, so its
     * temperature T* satisfies D C T* + sum_j rho_j u_j^2 = D C T + rho u^2.
     * (Taking T* = T would let the two-step relaxation create energy at the
     * rate sum_j rho_j |u_j - u|^2 (1/tau1 - 1/tau2), against the paper's
     * statement that the corrected equation conserves energy.) */
    double Tstar = s->literal_eq6 ? Tf : Tf - ediff / (D * C);
    for (int j = 0; j < ns; ++j) {
      double tau1 = s->tau1[(size_t)j * n + x], tau2 = s->tau2[(size_t)j * n + x];
      double feq[MAXQ], fst[MAXQ];
      equilibrium(D, Q, s->c, me.rho[j], s->M[j], me.u, Tf, feq);     /* Eq.(4) */
      equilibrium(D, Q, s->c, me.rho[j], s->M[j], uj[j], Tstar, fst); /* Eq.(6) */
      double w1 = 2.0 / (1.0 + 2.0 * tau1);
      for (int i = 0; i < Q; ++i) {
        double g = *pop(s, s->gpre, j, i, x);
        /* Eq.(24) */
        *pop(s, s->Gn, j, i, x) = g - w1 * (g - fst[i]) - w1 * (tau1 / tau2) * (fst[i] - feq[i]) +
                                  w1 * tau1 * S[j][i];
      }
    }
  }
  for (int x = 0; x < n; ++x) s->work += s->acc_node[x];  /* in node order */
}

/* 6. solid heat step, Eq.(45)-(47), and the interface source.
 * Reading (flux-matched form of Eq.(48)): the wall node's energy changes by
 * the reaction heat -dH r (Eq.(42)) minus the kinetic energy the diffusive
 * wall handed to the gas this step; conduction runs over solid face
 * neighbours only; faces on a closed domain edge are Dirichlet baths at T_bc
 * (or adiabatic where T_bc is NaN). */
static void solid(oracle_sim *s) {
  int n = s->n, D = s->D;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n; ++x) {
    s->acc_node[x] = 0.0;
    if (!(s->kind[x] == K_SOLID || s->kind[x] == K_WALL)) {
      s->Tsn[x] = s->Ts[x];
      continue;
    }
    double T = s->Ts[x], lap = 0.0, bflux = 0.0;
    for (int a = 0; a < D; ++a)
      for (int d = -1; d <= 1; d += 2) {
        int nb = face_nbr(s, x, a, d);
        if (nb < 0) {
          double tb = s->T_bc[2 * a + (d > 0)];
          if (!isnan(tb)) {
            lap += tb - T;
            bflux += tb - T;
          }
        } else if (s->kind[nb] == K_SOLID || s->kind[nb] == K_WALL) {
          lap += s->Ts[nb] - T;
        }
      }
    double Tn = T + s->alpha_s * lap;
    s->acc_node[x] = s->alpha_s * s->C_s * bflux;
    /* isothermal walls (prior art) exchange nothing with the solid */
    if (s->kind[x] == K_WALL && s->wall_mode == 0) {
      if (!s->eq48) {
        Tn += (s->wall_q[x] - s->wall_dE[x]) / s->C_s;
      } else {
        /* Eq.(48): the third term is the heat the gas next to the wall
         * exchanges with it, alpha^f rho^f c_p^f / (rho^s c_p^s) (T^f - T^s)
         * = kappa_f (T^f - T^s) / C_s per gas face neighbour, with the gas
         * conductivity kappa_f = sum_j (D+2) tau1_j C_j T / (2 M_j Pr_j)
         * (reading of the Prandtl number's kappa) at that neighbour.
         * Reading: the sign that makes heat flow from the warmer side (the
         * printed minus would move it up the gradient). */
        double qf = 0.0;
        for (int a = 0; a < D; ++a)
          for (int d = -1; d <= 1; d += 2) {
            int nb = face_nbr(s, x, a, d);
            if (nb < 0 || !gaslike(s, nb)) continue;
            double kap = 0.0;
            for (int j = 0; j < s->ns; ++j)
              kap += (D + 2.0) * s->tau1[(size_t)j * n + nb] * (s->rho[(size_t)j * n + nb] / s->M[j]) *
                     s->T[nb] / (2.0 * s->M[j] * s->Pr_j[j]);
            qf += kap * (s->T[nb] - T);
          }
        Tn += (s->wall_q[x] + qf) / s->C_s;
      }
    }
    s->Tsn[x] = Tn;
  }
  for (int x = 0; x < n; ++x) s->bheat += s->acc_node[x];  /* in node order */
}

/* 6b. Crank-Nicolson variant of the solid step (Sec. 5, recommended for
 * alpha_s > 1/(2D)): the Laplacian (with the Dirichlet faces) averaged over
 * the old and new temperature, the wall sources explicit,
 *   T' - (a/2) L T' = T + (a/2) L T + (Q_rxn - dE_gas)/C_s,
 * solved by Jacobi sweeps until no node changes by more than 2.5e-16 (1 + |T'|);
 * boundary heat alpha_s C_s times the mean of the old and new face fluxes. */
static double solid_lap(const oracle_sim *s, const double *T, int x, double *bflux, int *cnt,
                        double *nbsum, double *bcsum) {
  double lap = 0.0;
  *bflux = 0.0;
  *cnt = 0;
  *nbsum = 0.0;
  *bcsum = 0.0;
  for (int a = 0; a < s->D; ++a)
    for (int d = -1; d <= 1; d += 2) {
      int nb = face_nbr(s, x, a, d);
      if (nb < 0) {
        double tb = s->T_bc[2 * a + (d > 0)];
        if (!isnan(tb)) {
          lap += tb - T[x];
          *bflux += tb - T[x];
          *bcsum += tb;
          ++*cnt;
        }
      } else if (s->kind[nb] == K_SOLID || s->kind[nb] == K_WALL) {
        lap += T[nb] - T[x];
        *nbsum += T[nb];
        ++*cnt;
      }
    }
  return lap;
}

static void solid_cn(oracle_sim *s) {
  int n = s->n;
  double a = s->alpha_s;
  double *rhs = malloc((size_t)n * sizeof(double));
  double *X = malloc((size_t)n * sizeof(double));
  double *Y = malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n; ++x) {
    X[x] = s->Ts[x];
    rhs[x] = s->Ts[x];
    s->acc_node[x] = 0.0;
    if (!(s->kind[x] == K_SOLID || s->kind[x] == K_WALL)) continue;
    double bf, nbs, bcs;
    int cnt;
    double lap = solid_lap(s, s->Ts, x, &bf, &cnt, &nbs, &bcs);
    rhs[x] = s->Ts[x] + 0.5 * a * lap;
    if (s->kind[x] == K_WALL && s->wall_mode == 0) rhs[x] += (s->wall_q[x] - s->wall_dE[x]) / s->C_s;
    s->acc_node[x] = 0.5 * a * s->C_s * bf;
  }
  for (int x = 0; x < n; ++x) s->bheat += s->acc_node[x];
  for (int it = 0; it < 1000000; ++it) {
    double dmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : dmax)
    for (int x = 0; x < n; ++x) {
      Y[x] = X[x];
      if (!(s->kind[x] == K_SOLID || s->kind[x] == K_WALL)) continue;
      double bf, nbs, bcs;
      int cnt;
      (void)solid_lap(s, X, x, &bf, &cnt, &nbs, &bcs);
      Y[x] = (rhs[x] + 0.5 * a * (nbs + bcs)) / (1.0 + 0.5 * a * cnt);
      double dd = fabs(Y[x] - X[x]) / (1.0 + fabs(Y[x]));
      if (dd > dmax) dmax = dd;
    }
    double *t = X;
    X = Y;
    Y = t;
    if (dmax <= 2.5e-16) break; /* a couple of ulps: the fixed point in FP64 */
  }
#pragma omp parallel for schedule(static)
  for (int x = 0; x < n; ++x) {
    s->Tsn[x] = X[x];
    s->acc_node[x] = 0.0;
    if (!(s->kind[x] == K_SOLID || s->kind[x] == K_WALL)) continue;
    double bf, nbs, bcs;
    int cnt;
    (void)solid_lap(s, X, x, &bf, &cnt, &nbs, &bcs);
    s->acc_node[x] = 0.5 * a * s->C_s * bf;
  }
  for (int x = 0; x < n; ++x) s->bheat += s->acc_node[x];
  free(rhs);
  free(X);
  free(Y);
}

/* 7. inlet (equilibrium at the prescribed state, velocity of the first
 * interior plane) and outlet, reading for Sec. 6: equilibrium at the inlet
 * pressure with the mole fractions, temperature and velocity of the last
 * interior plane (zero gradient of those; a zero-gradient copy of the whole
 * state would leave the outlet pressure free, and a body-force-driven flow
 * then drains the domain and accelerates without bound). */
static void inlet_outlet(oracle_sim *s) {
  if (!s->inout) return;
  int n = s->n, Q = s->Q, nx = s->nx;
  double Cin = s->p_in / s->T_in;
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y) {
      int src = node_of(s, 2, y, z);
      double u[3] = {0, 0, 0};
      if (gaslike(s, src))
        for (int a = 0; a < 3; ++a) u[a] = s->u[(size_t)a * n + src];
      for (int xg = 0; xg < 2; ++xg) {
        int g = node_of(s, xg, y, z);
        for (int j = 0; j < s->ns; ++j) {
          double f[MAXQ];
          equilibrium(s->D, Q, s->c, s->M[j] * s->X_in[j] * Cin, s->M[j], u, s->T_in, f);
          for (int i = 0; i < Q; ++i) *pop(s, s->Gn, j, i, g) = f[i];
        }
      }
      int last = node_of(s, nx - 3, y, z);
      double ul[3], Cl = 0.0, Tl = s->T[last];
      for (int a = 0; a < 3; ++a) ul[a] = s->u[(size_t)a * n + last];
      for (int j = 0; j < s->ns; ++j) Cl += s->rho[(size_t)j * n + last] / s->M[j];
      double Cout = s->p_in / Tl;
      for (int xg = nx - 2; xg < nx; ++xg) {
        int g = node_of(s, xg, y, z);
        for (int j = 0; j < s->ns; ++j) {
          double Xj = s->rho[(size_t)j * n + last] / s->M[j] / Cl;
          double f[MAXQ];
          equilibrium(s->D, Q, s->c, s->M[j] * Xj * Cout, s->M[j], ul, Tl, f);
          for (int i = 0; i < Q; ++i) *pop(s, s->Gn, j, i, g) = f[i];
        }
      }
    }
}

int oracle_step(oracle_sim *s, int64_t n_steps) {
  if (!s || !s->init_done) return fail(s, "fields not initialised");
  for (int64_t t = 0; t < n_steps; ++t) {
    stream_all(s);
    wall_bc(s);
    moments(s);
    collide(s);
    if (s->solid_scheme == 1) solid_cn(s);
    else solid(s);
    inlet_outlet(s);
    for (int w = 0; w < s->n; ++w)
      if (s->kind[w] == K_WALL) {
        s->moles += s->wall_r[w];
        s->heat += s->wall_q[w];
      }
    double *t1 = s->G;
    s->G = s->Gn;
    s->Gn = t1;
    double *t2 = s->Ts;
    s->Ts = s->Tsn;
    s->Tsn = t2;
    s->step++;
  }
  return 0;
}

int oracle_observe(oracle_sim *s, oracle_obs *o) {
  if (!s || !o) return fail(s, "null argument");
  memset(o, 0, sizeof *o);
  int n = s->n, Q = s->Q;
  o->T_min = o->Ts_min = o->rho_min = DBL_MAX;
  o->T_max = o->Ts_max = -DBL_MAX;
  for (int x = 0; x < n; ++x) {
    int k = s->kind[x];
    if (k == K_SOLID || k == K_WALL) {
      o->n_solid++;
      o->e_solid += s->C_s * s->Ts[x];
      if (s->Ts[x] < o->Ts_min) o->Ts_min = s->Ts[x];
      if (s->Ts[x] > o->Ts_max) o->Ts_max = s->Ts[x];
      if (!isfinite(s->Ts[x]) || s->Ts[x] <= 0) o->bad = 1;
    }
    if (k == K_WALL) o->n_wall++;
    if (!(gaslike(s, x) || k == K_WALL)) continue;
    if (gaslike(s, x)) o->n_gas++;
    double rhot = 0.0, E = 0.0, C = 0.0, J[3] = {0, 0, 0};
    for (int j = 0; j < s->ns; ++j) {
      double rj = 0.0;
      for (int i = 0; i < Q; ++i) {
        if (k == K_WALL && !emits(s, x, i)) continue;
        double g = *pop(s, s->G, j, i, x);
        double c2 = (double)(s->c[i][0] * s->c[i][0] + s->c[i][1] * s->c[i][1] +
                             s->c[i][2] * s->c[i][2]);
        rj += g;
        E += s->cj[j] * s->cj[j] * c2 * g;
        for (int a = 0; a < 3; ++a) J[a] += s->cj[j] * s->c[i][a] * g;
        if (!isfinite(g)) o->bad = 1;
      }
      o->mass[j] += rj;
      if (gaslike(s, x)) {
        rhot += rj;
        C += rj / s->M[j];
        if (rj < o->rho_min) o->rho_min = rj;
      }
    }
    o->e_gas += 0.5 * E;
    if (gaslike(s, x)) {
      double u2 = (J[0] * J[0] + J[1] * J[1] + J[2] * J[2]) / (rhot * rhot);
      double T = (E - rhot * u2) / (s->D * C);
      if (T < o->T_min) o->T_min = T;
      if (T > o->T_max) o->T_max = T;
      if (sqrt(u2) > o->u_max) o->u_max = sqrt(u2);
      if (!(T > 0) || !(rhot > 0)) o->bad = 1;
    }
  }
  if (o->rho_min < 0) o->bad = 1;
  o->moles_reacted = s->moles;
  o->heat_released = s->heat;
  o->heat_boundary = s->bheat;
  o->work_body = s->work;
  o->step = s->step;
  return 0;
}

/* Fields of the last completed step.  RHO (species comp), U (axis comp) and
 * T are the moments of f computed in that step (pass-1 values: species
 * densities, mixture velocity, temperature before the source energy) at gas
 * nodes, and the wall state at wall nodes.  TS, POP (species comp, Q*n
 * values, the stored post-collision populations), KIND, WALL_R, WALL_DE. */
int oracle_get_field(oracle_sim *s, int field, int comp, double *dst) {
  if (!s || !dst) return fail(s, "null argument");
  int n = s->n, Q = s->Q;
  switch (field) {
    case OF_RHO:
      if (comp < 0 || comp >= s->ns) return fail(s, "bad species");
      for (int x = 0; x < n; ++x)
        dst[x] = (gaslike(s, x) || s->kind[x] == K_WALL) ? s->rho[(size_t)comp * n + x] : 0.0;
      return 0;
    case OF_U:
      if (comp < 0 || comp > 2) return fail(s, "bad axis");
      for (int x = 0; x < n; ++x)
        dst[x] = (gaslike(s, x) || s->kind[x] == K_WALL) ? s->u[(size_t)comp * n + x] : 0.0;
      return 0;
    case OF_T:
      for (int x = 0; x < n; ++x) dst[x] = (gaslike(s, x) || s->kind[x] == K_WALL) ? s->T[x] : 0.0;
      return 0;
    case OF_TS:
      for (int x = 0; x < n; ++x) dst[x] = (s->kind[x] == K_SOLID || s->kind[x] == K_WALL) ? s->Ts[x] : 0.0;
      return 0;
    case OF_POP:
      if (comp < 0 || comp >= s->ns) return fail(s, "bad species");
      memcpy(dst, &s->G[(size_t)comp * Q * n], sizeof(double) * (size_t)Q * n);
      return 0;
    case OF_KIND:
      for (int x = 0; x < n; ++x) dst[x] = s->kind[x];
      return 0;
    case OF_WALL_R:
      for (int x = 0; x < n; ++x) dst[x] = s->kind[x] == K_WALL ? s->wall_r[x] : 0.0;
      return 0;
    case OF_WALL_DE:
      for (int x = 0; x < n; ++x) dst[x] = s->kind[x] == K_WALL ? s->wall_dE[x] : 0.0;
      return 0;
  }
  return fail(s, "unknown field");
}

/* Temperature of the auxiliary equilibrium f*: 0 (default) the reading that
 * holds the mixture energy fixed, 1 the printed Eq.(6), f* at the mixture
 * temperature T (for comparing the two). */
int oracle_set_literal_eq6(oracle_sim *s, int on) {
  if (!s) return fail(s, "null simulation");
  s->literal_eq6 = on != 0;
  return 0;
}

/* Threads of the node loops (OpenMP; every sum runs in node order, so the
 * results do not depend on the count).  Returns the count in use. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* Solid-gas coupling at wall nodes: 0 (default) flux-matched, 1 Eq.(48) */
int oracle_set_coupling(oracle_sim *s, int eq48) {
  if (!s) return fail(s, "null simulation");
  if (eq48 && s->solid_scheme == 1) return fail(s, "Eq.(48) coupling with the forward-Euler solid only");
  s->eq48 = eq48 != 0;
  return 0;
}

/* Rate per wall node (0, the default, as in Sec. 4.3) or per unit wetted
 * wall area (1, the reading for sphere packs). */
int oracle_set_source_flux(oracle_sim *s, int on) {
  if (!s) return fail(s, "null simulation");
  s->src_flux = on != 0;
  return 0;
}

int oracle_set_rate_area(oracle_sim *s, int on) {
  if (!s) return fail(s, "null simulation");
  s->rate_area = on != 0;
  return 0;
}

int oracle_set_wall_position(oracle_sim *s, int halfway) {
  if (!s) return fail(s, "null simulation");
  if (halfway != 0 && halfway != 1) return fail(s, "wall position must be 0 (on the node) or 1 (half-way)");
  s->halfway = halfway;
  return 0;
}

/* Checkpoint: everything a later step or observation reads -- populations
 * (gas and wall slots), solid temperature, the last step's node fields
 * (densities, velocity, temperature, wall rate and energy exchange) and the
 * cumulative counters -- as one flat block of doubles.  A restored run
 * continues bitwise like the uninterrupted one. */
static size_t state_doubles(const oracle_sim *s) {
  const size_t n = (size_t)s->n;
  return (size_t)s->ns * s->Q * n + n + (size_t)s->ns * n + 3 * n + n + 2 * n + 5;
}

size_t oracle_state_bytes(const oracle_sim *s) { return s ? state_doubles(s) * sizeof(double) : 0; }

static void state_copy(oracle_sim *s, double *buf, int save) {
  const size_t n = (size_t)s->n;
  double *p = buf;
  struct {
    double *a;
    size_t len;
  } parts[] = {{s->G, (size_t)s->ns * s->Q * n}, {s->Ts, n}, {s->rho, (size_t)s->ns * n},
               {s->u, 3 * n}, {s->T, n}, {s->wall_r, n}, {s->wall_dE, n}};
  for (size_t k = 0; k < sizeof parts / sizeof parts[0]; ++k) {
    if (save) memcpy(p, parts[k].a, parts[k].len * sizeof(double));
    else memcpy(parts[k].a, p, parts[k].len * sizeof(double));
    p += parts[k].len;
  }
  if (save) {
    p[0] = s->moles;
    p[1] = s->heat;
    p[2] = s->bheat;
    p[3] = s->work;
    p[4] = (double)s->step;
  } else {
    s->moles = p[0];
    s->heat = p[1];
    s->bheat = p[2];
    s->work = p[3];
    s->step = (int64_t)p[4];
  }
}

int oracle_save_state(oracle_sim *s, void *dst, size_t bytes) {
  if (!s || !dst) return fail(s, "null argument");
  if (!s->init_done) return fail(s, "initialise the fields first");
  if (bytes < oracle_state_bytes(s)) return fail(s, "checkpoint buffer too small");
  state_copy(s, (double *)dst, 1);
  return 0;
}

int oracle_load_state(oracle_sim *s, const void *src, size_t bytes) {
  if (!s || !src) return fail(s, "null argument");
  if (!s->init_done) return fail(s, "initialise the fields first");
  if (bytes != oracle_state_bytes(s)) return fail(s, "checkpoint of another size");
  state_copy(s, (double *)src, 0);
  return 0;
}

/* Overwrite the populations of species comp (Q*n values, the layout of
 * oracle_get_field's OF_POP): a building block for the linear stability
 * analysis, which needs arbitrary, not only equilibrium, states. */
int oracle_set_pops(oracle_sim *s, int comp, const double *src) {
  if (!s || !src) return fail(s, "null argument");
  if (!s->init_done) return fail(s, "initialise the fields first");
  if (comp < 0 || comp >= s->ns) return fail(s, "bad species");
  memcpy(&s->G[(size_t)comp * s->Q * s->n], src, sizeof(double) * (size_t)s->Q * s->n);
  return 0;
}

/* Third-moment and energy-flux deviations of the lattice equilibrium from the
 * Maxwellian at a state (exposed for the pin tests): Qaaa[3] = Q'_aaa,
 * *Qxyz = Q'_xyz (3-D), R9[3a+b] = R'_ab, all in physical units of species j. */
int oracle_deviations(int lattice, double rho_j, double M_j, const double *u3, double T,
                      double *Qaaa, double *Qxyz, double *R9) {
  oracle_sim tmp;
  memset(&tmp, 0, sizeof tmp);
  if (lattice != 2 && lattice != 3) return -1;
  tmp.D = lattice;
  tmp.M[0] = M_j;
  nbstate v;
  memset(&v, 0, sizeof v);
  v.rho[0] = rho_j;
  v.T = T;
  for (int a = 0; a < 3; ++a) v.u[a] = a < lattice ? u3[a] : 0.0;
  for (int a = 0; a < 3; ++a) Qaaa[a] = a < lattice ? Qdev_aaa(&tmp, 0, &v, a) : 0.0;
  *Qxyz = lattice == 3 ? Qdev_xyz(0, &v) : 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) R9[3 * a + b] = (a < lattice && b < lattice) ? Rdev(&tmp, 0, &v, a, b) : 0.0;
  return 0;
}
