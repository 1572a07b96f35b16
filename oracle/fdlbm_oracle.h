/*
 * FP64 CPU oracle of the coupled FD-LBM step (Kulyk, Berger, Smith, Harting,
 * "Catalytic flow with a coupled Finite Difference - Lattice Boltzmann scheme").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct reference
 * used by the tests and by the benchmark's CPU-baseline leg.  The product (the
 * HIP library) never links, loads or calls it, and it shares no code, header or
 * table with the product.
 *
 * Everything is double precision, plain nested loops over nodes (split over
 * OpenMP threads where the nodes are independent; every sum in node order).  Equation
 * numbers refer to the paper in the order of its display equations:
 *   Eq.(1)  two-step BGK kinetic equation          Eq.(2)  species lattice velocities
 *   Eq.(4)  mixture equilibrium                     Eq.(5)  mixture moments
 *   Eq.(6)  auxiliary equilibrium f*                Eq.(7-8) tau2, mixture diffusion
 *   Eq.(11) diffusion-velocity correction U^c       Eq.(12-13) its forcing, psi vectors
 *   Eq.(14-17) Wilke viscosity, tau1                Eq.(19-21) Prandtl correction
 *   Eq.(23) g-transform   Eq.(24) trapezoidal collision   Eq.(25) f-moments from g
 *   Eq.(33-36) off-lattice streaming interpolation  Eq.(37-41) reactive diffusive wall
 *   Eq.(42) reaction enthalpy   Eq.(46-48) solid FD heat step and interface
 *   Eq.(50) surface rate law
 */
#ifndef FDLBM_ORACLE_H
#define FDLBM_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAXS 8
#define ORACLE_MAXR 4 /* surface reactions */

typedef struct oracle_sim oracle_sim;

typedef struct {
  double mass[ORACLE_MAXS];   /* per-species gas mass incl. wall-emitted pops in flight */
  double e_gas;               /* (1/2) sum c^2 g over gas pops and wall-emitted pops    */
  double e_solid;             /* sum C_s T^s over solid nodes                            */
  double moles_reacted;       /* cumulative sum over steps and wall nodes of r_w          */
  double heat_released;       /* cumulative -dH * r_w                                     */
  double heat_boundary;       /* cumulative heat into the solid through Dirichlet faces   */
  double work_body;           /* cumulative work of the body force on the gas             */
  double T_min, T_max, u_max, rho_min;
  double Ts_min, Ts_max;
  int64_t step;
  int32_t bad;                /* 1 if a NaN/Inf, negative density or temperature seen   */
  int32_t n_gas, n_wall, n_solid;
} oracle_obs;

/* lattice: 2 = D2Q9, 3 = D3Q19.  periodic[a] nonzero: axis a wraps.
 * inout: 1 = planes x=0,1 are inlet ghosts and x=nx-2,nx-1 outlet ghosts. */
oracle_sim *oracle_create(int lattice, int nx, int ny, int nz, const int *periodic,
                          int n_species);
void oracle_destroy(oracle_sim *s);
const char *oracle_error(const oracle_sim *s);

int oracle_set_geometry(oracle_sim *s, const uint8_t *mask, int inout);
int oracle_set_species(oracle_sim *s, const double *M, const double *mu0, double mu_T_exp,
                       const double *Djk0, double D_T_exp, double D_p_exp, double T_ref,
                       double p_ref, double Pr, unsigned flags);
/* flags: 1 diffusion velocity, 2 viscous, 4 energy-flux, 8 Prandtl
 * corrections; diagnostic bits for the pin tests: 16 drops the cubic Q'_xyz
 * part of the viscous correction, 32 the off-diagonal R'_ab of the energy-flux
 * correction */
/* per-species Prandtl numbers (NULL: every species at the common Pr) */
int oracle_set_prandtl(oracle_sim *s, const double *Pr_j);
/* Lennard-Jones transport from a collision-integral table (NULL eps: off) */
int oracle_set_lj(oracle_sim *s, const double *eps_over_k, double T_unit, double tmin, double tmax, int n,
                  const double *om_mu, const double *om_d);
int oracle_set_solid(oracle_sim *s, double alpha_s, double C_s, const double *T_bc6);
/* solid time scheme: 0 forward Euler (alpha_s <= 1/(2D)), 1 Crank-Nicolson */
int oracle_set_solid_scheme(oracle_sim *s, int scheme);
int oracle_set_reaction(oracle_sim *s, const double *nu, const double *order, double k0,
                        double ea, double T_ref, double dH, int wall_mode, double T_iso,
                        double tol, int max_iter);
/* wall velocity U_w of Eq.(39) per node (u3[a*n + node], read at wall
 * nodes; NULL: walls at rest, the default): the diffusive wall then emits
 * rho_w f^eq(1, U_w, T_w) and its state seen by the gradients moves */
int oracle_set_wall_velocity(oracle_sim *s, const double *u3);
int oracle_set_flow(oracle_sim *s, const double *F3, const double *X_in, double p_in,
                    double T_in);
/* rho[j*n + node], u[a*n + node] (3 rows), T[n], Ts[n]; populations set to f^eq. */
int oracle_init_fields(oracle_sim *s, const double *rho, const double *u, const double *T,
                       const double *Ts);
int oracle_step(oracle_sim *s, int64_t n_steps);
int oracle_observe(oracle_sim *s, oracle_obs *out);

/* field ids for oracle_get_field (dst holds n doubles, POP holds Q*n) */
enum { OF_RHO = 0, OF_U = 1, OF_T = 2, OF_TS = 3, OF_POP = 4, OF_KIND = 5, OF_WALL_R = 6,
       OF_WALL_DE = 7 };
int oracle_get_field(oracle_sim *s, int field, int comp, double *dst);
/* threads of the node loops (<= 0: keep); returns the count in use */
int oracle_set_threads(int n);
/* solid-gas coupling at wall nodes: 0 flux-matched (default), 1 Eq.(48) */
int oracle_set_coupling(oracle_sim *s, int eq48);
/* reaction rate per wall node (0, default) or per unit wetted area (1) */
int oracle_set_rate_area(oracle_sim *s, int on);
/* a further surface reaction (stoichiometry, orders, k0, E_a/(R T_ref),
 * T_ref, dH) after the one of oracle_set_reaction, up to ORACLE_MAXR in all;
 * every wall node runs all of them (reading) */
int oracle_add_reaction(oracle_sim *s, const double *nu, const double *order, double k0, double ea,
                        double T_ref, double dH);
/* wall source in population units: nu_j M_j r (0, default) or nu_j M_j r / c_j (1) */
int oracle_set_source_flux(oracle_sim *s, int on);
/* wall position: on the solid node (0, default, Eq.(39)) or half-way along
 * each link (1): the wall node emits at the state extrapolated through the
 * link's midpoint from the gas node it emits into (Sec. 4.3, reading) */
int oracle_set_wall_position(oracle_sim *s, int halfway);
/* f* temperature: 0 the energy-holding reading (default), 1 Eq.(6) as printed */
int oracle_set_literal_eq6(oracle_sim *s, int on);
/* overwrite the populations of species comp (Q*n values, OF_POP layout) */
int oracle_set_pops(oracle_sim *s, int comp, const double *src);
/* checkpoint of the state (populations, solid temperature, last node fields,
 * counters): size, save into dst, restore from src (same geometry) */
size_t oracle_state_bytes(const oracle_sim *s);
int oracle_save_state(oracle_sim *s, void *dst, size_t bytes);
int oracle_load_state(oracle_sim *s, const void *src, size_t bytes);

/* ---- building blocks exposed for the pin tests ---- */
/* equilibrium populations of one species, Eq.(4)/(6) (D2Q9) or the D3Q19 reading */
int oracle_equilibrium(int lattice, double rho_j, double M_j, const double *u3, double T,
                       double *f_out);
/* source shapes: which = 0 psi_x, 1 psi_y, 2 psi_z, 3..8 pi_xx,yy,zz,xy,xz,yz,
 * 9..11 chi_x,y,z, 12 phi (energy); unscaled (c_j = 1) */
int oracle_shape(int lattice, int which, double *out);
/* Lagrange weights of stencil class k (0..6) at shift s, taps at t = offsets */
int oracle_interp_weights(int cls, double s, double *w3, int *t3, int *ntaps);
/* lattice velocity table (c[i*3+a]), returns Q */
int oracle_velocities(int lattice, int *c_out);
/* lattice-minus-Maxwellian third moments Q'_aaa, Q'_xyz and energy flux R'_ab */
int oracle_deviations(int lattice, double rho_j, double M_j, const double *u3, double T,
                      double *Qaaa, double *Qxyz, double *R9);
/* transport at a state: tau1[j], tau2[j] (Eq.(7-8), (14-17)) */
int oracle_transport(oracle_sim *s, const double *rho, double T, double *tau1, double *tau2);

#ifdef __cplusplus
}
#endif
#endif
