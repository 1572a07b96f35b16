/*
 * fdlbm.h -- C ABI of the MI355X (gfx950) implementation of the coupled
 * finite-difference / lattice-Boltzmann step for catalytic reactive flow
 * (Kulyk, Berger, Smith, Harting, "Catalytic flow with a coupled Finite
 * Difference - Lattice Boltzmann scheme").
 *
 * One time step advances
 *   - the gas: Kang et al.'s thermal multicomponent LBM, one population set per
 *     species with species lattice speeds c_j = sqrt(M_0/M_j) (Eq.(2)), pull
 *     streaming with the off-lattice interpolation of Eq.(33)-(36), the
 *     two-step BGK collision in its trapezoidal form Eq.(24) with the moments
 *     of Eq.(25), and the correction sources of Sec. 3 (diffusion velocity
 *     Eq.(11)-(13), Prandtl number Eq.(19)-(21), lattice-deviation terms);
 *   - the reactive diffusive wall on the solid nodes, Eq.(37)-(41) with the
 *     rate law Eq.(50) and the reaction enthalpy Eq.(42);
 *   - the solid: heat equation Eq.(45)-(47) by forward Euler (or, as an
 *     option, Crank-Nicolson) coupled at the wall nodes (Eq.(48),
 *     flux-matched form).
 *
 * Units: lattice units.  Masses relative to the lightest species (>= 1);
 * the reference temperature is 1/3; pressure p = C T with C = sum rho_j/M_j.
 *
 * Memory: the caller allocates ONE device buffer (e.g. a torch tensor) of
 * fdlbm_workspace_bytes() bytes, 256-byte aligned, and binds it; the library
 * allocates no device memory of its own and never frees the caller's buffer.
 * All kernels run on the stream given at creation (NULL = default stream).
 * Host arrays passed in are copied before the call returns.
 *
 * Errors: every int-returning call returns FDLBM_OK (0) or a negative code;
 * fdlbm_last_error() gives a message.  No exception crosses the ABI.
 * Thread-compatible: one context per host thread.
 *
 * Layouts: node index = x + nx*(y + ny*z).  Host arrays are per node; the
 * workspace stores populations per (direction, slot) as records of all
 * species and moments as per-slot records (slots: gas nodes, then wall
 * nodes), and fdlbm_get_field returns populations of species j, direction i
 * at [i*n + node] (structure of arrays, zero where a node stores none).  Direction
 * order: D2Q9 as Eq.(2) (rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1));
 * D3Q19 rest, +x, -x, +y, -y, +z, -z, then the xy, xz, yz edges, each in the
 * order (+,+), (-,+), (-,-), (+,-).
 */
#ifndef FDLBM_H
#define FDLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FDLBM_OK 0
#define FDLBM_E_INVALID -1   /* bad argument or parameter out of range        */
#define FDLBM_E_GEOMETRY -2  /* mask rejected (no gas, gas on a closed edge)  */
#define FDLBM_E_ALIGN -3     /* workspace too small or not 256-byte aligned   */
#define FDLBM_E_HIP -4       /* a HIP runtime call failed                     */
#define FDLBM_E_UNSTABLE -5  /* NaN/Inf, negative density or temperature seen  */
#define FDLBM_E_STATE -6     /* call made out of order                        */

/* lattices and precisions */
#define FDLBM_D2Q9 2
#define FDLBM_D3Q19 3
#define FDLBM_F64 0
#define FDLBM_F32 1
#define FDLBM_F16 2   /* populations stored as FP16 g/rho_ref,j - w_i; FP32 arithmetic */
#define FDLBM_BF16 3  /* populations stored as BF16 g/rho_ref,j - w_i; FP32 arithmetic */

/* correction-term switches (Sec. 3 / Sec. 4.1) */
#define FDLBM_CORR_DIFFUSION 1u  /* diffusion-velocity correction, Eq.(11)-(13)  */
#define FDLBM_CORR_VISCOUS 2u    /* third-moment lattice-deviation correction    */
#define FDLBM_CORR_ENERGY 4u     /* energy-flux lattice-deviation correction     */
#define FDLBM_CORR_PRANDTL 8u    /* variable Prandtl number, Eq.(19)-(21)        */
#define FDLBM_CORR_ALL 15u
/* The energy-flux correction's heat-conduction part and the Prandtl
 * correction add heat diffusion explicitly (as energy sources in face-flux
 * form), which bounds the relaxation times: with Pr = 1 the step is
 * linearly stable for tau1 below 1/2 (the checkerboard mode is multiplied
 * by 1 - 4 tau1 on D3Q19); the Prandtl term tightens this for Pr < 1
 * (single species, Pr = 0.71: stable at tau1 = 0.1 on D3Q19 and 0.45 on
 * D2Q9).  The packed bed's mixture is stable.  A run beyond the bound
 * blows up; fdlbm_set_sync_check reports it. */

/* wall modes */
#define FDLBM_WALL_REACTIVE 0   /* T_w = solid temperature, heat exchanged (Sec. 5) */
#define FDLBM_WALL_ISOTHERMAL 1 /* fixed T_w, no exchange with the solid (prior art) */

/* field ids for fdlbm_get_field */
#define FDLBM_FIELD_RHO 0     /* species density (comp = species)              */
#define FDLBM_FIELD_U 1       /* mixture velocity (comp = axis)                */
#define FDLBM_FIELD_T 2       /* gas temperature                               */
#define FDLBM_FIELD_TS 3      /* solid temperature                             */
#define FDLBM_FIELD_POP 4     /* stored populations of species comp (Q*n)      */
#define FDLBM_FIELD_KIND 5    /* node class: 0 gas 1 solid 2 wall 3 inlet 4 outlet */
#define FDLBM_FIELD_WALL_R 6  /* molar rate per wall node in the last step      */
#define FDLBM_FIELD_WALL_DE 7 /* kinetic energy the wall gave the gas, last step */
#define FDLBM_FIELD_X 8       /* mole fraction (comp = species), Eq.(14)        */

#define FDLBM_MAX_SPECIES 8

typedef struct fdlbm_ctx fdlbm_ctx;

typedef struct {
  int lattice;      /* FDLBM_D2Q9 or FDLBM_D3Q19                                 */
  int nx, ny, nz;   /* grid; nz = 1 for D2Q9                                    */
  int periodic[3];  /* nonzero: axis wraps                                      */
  int precision;    /* FDLBM_F64, FDLBM_F32 (storage and arithmetic), or         *
                     * FDLBM_F16 / FDLBM_BF16 (16-bit population storage, FP32   *
                     * arithmetic and every other field FP32)                    */
  int n_species;    /* 1 .. FDLBM_MAX_SPECIES                                   */
  void *hip_stream; /* hipStream_t to run on; NULL = default stream             */
} fdlbm_desc;

typedef struct {
  double mass[FDLBM_MAX_SPECIES]; /* per-species gas mass incl. wall-emitted pops */
  double e_gas;          /* (1/2) sum_j sum_i c_ji^2 g over gas + wall-emitted pops */
  double e_solid;        /* sum over solid nodes of C_s T^s                         */
  double moles_reacted;  /* cumulative reaction extent, sum over steps and walls    */
  double heat_released;  /* cumulative -dH * moles_reacted (Eq.(42))               */
  double heat_boundary;  /* cumulative heat into the solid through Dirichlet faces */
  double work_body;      /* cumulative work of the body force on the gas          */
  double T_min, T_max, u_max, rho_min;
  double Ts_min, Ts_max;
  int64_t step;
  int32_t bad;           /* 1 if NaN/Inf, negative density or temperature seen    */
  int32_t n_gas, n_wall, n_solid;
} fdlbm_obs;

/* Create a context for one domain (no device memory yet): the lattice of
 * Sec. 2 (D2Q9 of Eq.(2), or the D3Q19 extension), the grid of lattice
 * units of Sec. 4.1 (one node per lattice spacing, one step per time step),
 * the number of gas species of the mixture and the precision.  *out owned
 * by the caller until fdlbm_destroy.  Errors: FDLBM_E_INVALID on bad sizes
 * or counts, and on more than 2^30 nodes (the kernels address node-indexed
 * tables with 32-bit byte offsets). */
int fdlbm_create(const fdlbm_desc *d, fdlbm_ctx **out);

/* Release the context (no step of the method).  Does not free the
 * caller's workspace. */
void fdlbm_destroy(fdlbm_ctx *ctx);

/* Message of the last error on this context (static storage of ctx). */
const char *fdlbm_last_error(const fdlbm_ctx *ctx);

/* Geometry (Sec. 4.3, wall on the first solid node): mask_host[n] with 0 =
 * gas, 1 = solid, copied.  Wall nodes are the solid nodes with a gas node
 * among their lattice neighbours.  inout = 1 turns the planes x = 0, 1 into
 * inlet nodes (equilibrium at the inlet state, Sec. 6) and x = nx-2, nx-1
 * into outlet nodes (equilibrium at the inlet pressure with the mole
 * fractions, temperature and velocity of x = nx-3); x must then be
 * non-periodic, those planes gas and x = nx-3 gas wherever the outlet is.
 * FDLBM_E_GEOMETRY if no gas node exists, a gas node touches a closed domain
 * edge or an outlet row has no interior gas node to copy; FDLBM_E_INVALID if
 * one direction's populations (gas and wall nodes times the stored record:
 * 4 bytes per species in FP32, 8 in FP64, 2 in 16-bit storage, rounded up to
 * an even count) would exceed 4 GiB, the span the population gathers
 * address with 32-bit offsets (FP32 with five species: about 214 million gas
 * and wall nodes, a 640^3 bed). */
int fdlbm_set_geometry(fdlbm_ctx *ctx, const uint8_t *mask_host, int inout);

/* Species and transport (Sec. 3, Eq.(7)-(8), (14)-(17), (19)-(21)):
 * M[j] relative masses (>= 1); mu0[j] viscosities at T_ref, mu_j = mu0_j
 * (T/T_ref)^mu_T_exp; Djk0[j*ns+k] symmetric binary diffusivities at
 * (T_ref, p_ref), D_jk = Djk0 (T/T_ref)^D_T_exp (p_ref/p)^D_p_exp; Pr the
 * Prandtl number; corr_flags a mask of FDLBM_CORR_*.  Copied. */
int fdlbm_set_species(fdlbm_ctx *ctx, const double *M, const double *mu0, double mu_T_exp,
                      const double *Djk0, double D_T_exp, double D_p_exp, double T_ref,
                      double p_ref, double Pr, unsigned corr_flags);

/* Per-species Prandtl numbers Pr_j (> 0, n_species values; NULL: every
 * species at the Pr of fdlbm_set_species, which also resets them).  The
 * Prandtl correction of Eq.(19)-(21) then uses q^Pr_j = (D+2)(1/Pr_j - 1)
 * tau1_j C_j T grad T / M_j for species j: the per-species extension Sec. 3
 * mentions after Eq.(21).  Call after fdlbm_set_species. */
int fdlbm_set_prandtl(fdlbm_ctx *ctx, const double *Pr_j);

/* Lennard-Jones transport, Eq.(26)-(27): the viscosities and binary
 * diffusivities take their temperature dependence from collision integrals
 * instead of power laws, scaled from the reference values of
 * fdlbm_set_species (mu0_j, Djk0 at T_ref, p_ref):
 *   mu_j   = mu0_j  (T/T_ref)^(1/2) Omega_mu(T*_ref,j) / Omega_mu(T*_j),
 *   D_jk   = Djk0   (T/T_ref)^(3/2) (p_ref/p) Omega_D(T*_ref,jk) / Omega_D(T*_jk),
 * T*_j = T T_unit / eps_j, eps_jk = sqrt(eps_j eps_k) (the "T^3" of Eq.(27)
 * read as T^(3/2)); Wilke's phi_jk (Eq.(15)) then follow the local
 * viscosities.  eps_over_k: n_species well depths (K); T_unit: kelvin per
 * lattice temperature unit; the table: n (2..64) values of Omega_mu and
 * Omega_D on a uniform grid of T* from tstar_min to tstar_max, interpolated
 * linearly and held constant beyond its ends (the caller supplies it, e.g.
 * from a published collision-integral table).  eps_over_k NULL: power laws
 * again.  Call after fdlbm_set_species; copied. */
int fdlbm_set_lj_transport(fdlbm_ctx *ctx, const double *eps_over_k, double T_unit, double tstar_min,
                           double tstar_max, int n, const double *omega_mu, const double *omega_d);

/* Solid (Eq.(45)-(47)): thermal diffusivity alpha_s (alpha_s >= 0; with the
 * forward-Euler scheme, the default, also alpha_s <= 1/(2D), its stability
 * bound; else FDLBM_E_INVALID), volumetric heat capacity
 * C_s > 0, and T_bc6[6] Dirichlet temperatures of the closed domain faces
 * (-x, +x, -y, +y, -z, +z; NaN = adiabatic; NULL = all adiabatic). */
int fdlbm_set_solid(fdlbm_ctx *ctx, double alpha_s, double C_s, const double *T_bc6);

/* Time scheme of the solid heat equation.  FDLBM_SOLID_EULER (default):
 * forward Euler, Eq.(46)-(47), stable for alpha_s <= 1/(2D).
 * FDLBM_SOLID_CN: Crank-Nicolson, the extension Sec. 5 recommends for larger
 * alpha_s: T' - (alpha_s/2) L T' = T + (alpha_s/2) L T + wall sources/C_s,
 * solved by Jacobi sweeps from T, as many as make the error bound
 * (a D / (1 + a D))^k fall below 1e-15 (FP64) or 1e-8 (FP32 arithmetic)
 * relative to the step (at most 5000); the Dirichlet-face heat is the mean
 * of the old and new face fluxes.  Choose CN before fdlbm_set_solid with
 * alpha_s > 1/(2D); switching back to Euler with such an alpha_s fails.
 * In a batch every sample uses the same scheme; Crank-Nicolson samples may
 * take different numbers of sweeps. */
#define FDLBM_SOLID_EULER 0
#define FDLBM_SOLID_CN 1
int fdlbm_set_solid_scheme(fdlbm_ctx *ctx, int scheme);

/* Solid-gas coupling at the wall nodes (Sec. 5, Eq.(48)).
 * FDLBM_COUPLING_FLUX (default): the wall node's solid energy changes by
 * the reaction heat (Eq.(42)) minus the kinetic energy the diffusive wall
 * handed the gas in the same step, so the interface conserves energy
 * exactly (the enthalpy error of Eq.(49) is rounding).
 * FDLBM_COUPLING_EQ48: Eq.(48) itself, the third term read with the sign
 * that moves heat from the warmer side: per gas face neighbour
 * kappa_f (T^f - T^s) / C_s with kappa_f = sum_j (D+2) tau1_j C_j T /
 * (2 M_j Pr_j) from that neighbour's moments of the step; the diffusive
 * wall still hands the gas its energy, so the interface does not conserve
 * energy (Eq.(49)'s error is then about 3 % on the channel workload) and
 * the solid step waits for the moments (no overlap).  Forward-Euler solid
 * only; in a batch every sample has the same coupling; FDLBM_E_INVALID
 * otherwise or for another value. */
#define FDLBM_COUPLING_FLUX 0
#define FDLBM_COUPLING_EQ48 1
int fdlbm_set_solid_coupling(fdlbm_ctx *ctx, int mode);

/* Surface reaction (Eq.(50) generalised): molar rate per wall node and step
 * r = k0 exp[ea (1 - T_ref/T_w)] prod_j C_jw^order_j, species j produced at
 * nu_j per unit extent (nu < 0 reactants); orders must be integers 0..3.
 * dH reaction enthalpy per unit extent (< 0 exothermic), Eq.(42).
 * wall_mode FDLBM_WALL_*; T_iso the wall temperature in isothermal mode;
 * tol / max_iter bound the wall-density fixed point of Sec. 4.3.  Replaces
 * every reaction set before (one reaction afterwards). */
int fdlbm_set_reaction(fdlbm_ctx *ctx, const double *nu, const double *order, double k0,
                       double ea, double T_ref, double dH, int wall_mode, double T_iso,
                       double tol, int max_iter);

/* A further surface reaction at every wall node, with the same arguments as
 * the rate law of fdlbm_set_reaction (nu, order: n_species values, copied).
 * Sec. 4.3 takes any source S_j in the flux balance of Eq.(38)-(41); with
 * several reactions S_j = sum_k nu_jk M_j r_k.  The wall-density fixed point
 * then updates every species some reaction consumes with a positive order,
 * each with its own consumption implicit and its production at the current
 * densities; the reaction heat at the node is sum_k -dH_k r_k (Eq.(42)),
 * FDLBM_FIELD_WALL_R and moles_reacted count the summed rates, and
 * heat_released sums the heat node by node.  Up to FDLBM_MAX_REACTIONS in
 * all.  FDLBM_E_STATE before fdlbm_set_reaction; FDLBM_E_INVALID beyond the
 * limit or for orders outside 0..3.  In a batch, either every sample or
 * none has several reactions.  Takes effect at the next step. */
#define FDLBM_MAX_REACTIONS 4
int fdlbm_add_reaction(fdlbm_ctx *ctx, const double *nu, const double *order, double k0, double ea,
                       double T_ref, double dH);

/* Scaling of the surface rate at a wall node.  FDLBM_RATE_PER_NODE (the
 * default): one reaction term S_j per wall node, also at corner nodes, as
 * Sec. 4.3 states for walls built from plane and convex corner nodes.
 * FDLBM_RATE_PER_AREA (a reading for geometries with concave corners, such
 * as sphere packs, which the paper excludes): the rate is a flux per unit
 * wall area, so each node's rate is multiplied by its wetted area, its rest
 * emission weight over the links into the gas relative to a plane wall's
 * T_w / 2 (1 on plane walls; summed over a staircase sphere it is 1.21 times
 * the sphere's area).  Per node, the one-link wall nodes of a sphere pack
 * emit their whole production through one link, and trace product
 * densities next to them turn negative within steps at k0 = 2e-3.
 * FDLBM_E_INVALID for another value.  Takes effect at the next step. */
#define FDLBM_RATE_PER_NODE 0
#define FDLBM_RATE_PER_AREA 1
int fdlbm_set_rate_scaling(fdlbm_ctx *ctx, int mode);

/* Population mass the reactive wall adds per unit of nu_j M_j r (Eq.(38)-(41)
 * with Eq.(50)).  FDLBM_SOURCE_LATTICE (the default): S_j / c_j = nu_j M_j r
 * (the flux sums of Eq.(38)-(39) taken with the species velocities c_j e_i
 * and S_j as Eq.(50) prints it).  FDLBM_SOURCE_FLUX: nu_j M_j r / c_j.  An
 * interpolated species (c_j < 1) moves a population c_j of a link per step,
 * so the mass the gas receives per step is the emitted excess times about
 * c_j: with the default the gas receives about c_j nu_j M_j r of species j
 * (a product of mass ratio 4 arrives about half short in a reactive channel),
 * with FDLBM_SOURCE_FLUX it receives nu_j M_j r after a start-up transient
 * (the stoichiometric product balance Sec. 7 reports).  On sphere packs the
 * 1/c_j larger emission at one-link wall nodes drives trace product densities
 * negative within steps; the default keeps them positive.  On-lattice species
 * (c_j = 1) are the same in both.  FDLBM_E_INVALID for another value.  Takes
 * effect at the next step. */
#define FDLBM_SOURCE_LATTICE 0
#define FDLBM_SOURCE_FLUX 1
int fdlbm_set_wall_source(fdlbm_ctx *ctx, int mode);

/* Where the diffusive wall sits (Sec. 4.3).  FDLBM_WALL_ON_NODE (the
 * default): on the wall node, which thermalises at its own state
 * f^eq(rho_w, 0, T_w) (Eq.(39)).  FDLBM_WALL_HALFWAY: half-way between the
 * wall node and each gas node it emits into; the paper names the extra
 * interpolation step this needs without giving it, and the reading here is
 * the linear one: along link i into gas node x the wall node emits
 * rho_w f^eq_i(1, -u(x), 2 T_w - T(x)), the state whose linear interpolant
 * with x takes the wall's velocity (zero) and temperature at the link's
 * midpoint, with u(x) and T(x) from x's moments of the previous step.  rho_w
 * still solves the mass balance of Eq.(41) with these weights, so mass and
 * energy stay conserved.  A Poiseuille channel's velocity zeros then sit half
 * a node from the wall nodes.  The moments pass then waits for the wall
 * kernel (which reads the moments it overwrites), so the step loses the wall
 * kernel's overlap.  In a batch every sample has the same wall position.
 * FDLBM_E_INVALID for another value.  Takes effect at the next step. */
#define FDLBM_WALL_ON_NODE 0
#define FDLBM_WALL_HALFWAY 1
int fdlbm_set_wall_position(fdlbm_ctx *ctx, int position);

/* Flow: body force per unit mass F3[3]; inlet mole fractions X_in[ns],
 * pressure p_in and temperature T_in (used when inout = 1). */
int fdlbm_set_flow(fdlbm_ctx *ctx, const double *F3, const double *X_in, double p_in,
                   double T_in);

/* Device bytes the caller must provide for the state of Sec. 4-5 (the
 * populations of every gas species and wall node, their moments, the solid
 * temperature; depends on the geometry: valid after fdlbm_set_geometry,
 * else FDLBM_E_STATE). */
int fdlbm_workspace_bytes(const fdlbm_ctx *ctx, size_t *bytes);

/* Bind the caller's device buffer (>= fdlbm_workspace_bytes, 256-byte
 * aligned, else FDLBM_E_ALIGN).  Requires the geometry; uploads it. */
int fdlbm_bind_workspace(fdlbm_ctx *ctx, void *dev_ptr, size_t bytes);

/* Initial state from host arrays: rho[j*n + node], u[a*n + node] (3 rows),
 * T[n], Ts[n].  Gas populations are set to f^eq (Eq.(4)); wall nodes emit
 * rho_w f^eq(1, 0, T_w) with rho_w the mean density of their gas partners.
 * Resets the step counter and the cumulative counters.  With 16-bit storage
 * it also fixes the reference densities rho_ref,j (mean initial density of
 * species j over the gas nodes, floored at 1e-12 of the total; kept in
 * checkpoints); the stored value of a population is g / rho_ref,j - w_i with
 * w_i the lattice weights at rest and T = 1/3.  FP16 overflows (the state
 * turns non-finite and fdlbm_observe reports it) if a species grows beyond
 * about 6e4 times its reference density. */
int fdlbm_init_fields(fdlbm_ctx *ctx, const double *rho, const double *u, const double *T,
                      const double *Ts);

/* Enqueue n_steps time steps on the context's stream (asynchronous).  One
 * step is the whole update of Sec. 4-5 in the paper's order: the reactive
 * wall (Eq.(37)-(42), (50)), streaming with the interpolation of
 * Eq.(33)-(36), moments and transport (Eq.(3), (5), (7)-(8), (14)-(17),
 * (25)), the correction sources (Eq.(11)-(13), (19)-(21)), the collision
 * (Eq.(4), (6), (24)), the solid heat step (Eq.(45)-(48)) and the
 * inlet/outlet planes (Sec. 6).
 * Every step also keeps a stability record on the device: the moments pass
 * marks the first step in which a gas node has a non-finite or negative
 * density or temperature.  With a check interval set (fdlbm_set_sync_check)
 * the call runs the steps in chunks of that many, synchronises after each
 * chunk, and returns FDLBM_E_UNSTABLE after the chunk in which the record
 * was set (the state then holds the end of that chunk; fdlbm_last_step
 * gives the step).  Without it the call only enqueues and returns FDLBM_OK.
 * Errors: FDLBM_E_STATE before fdlbm_init_fields, FDLBM_E_INVALID for a
 * negative count, FDLBM_E_HIP if a launch fails. */
int fdlbm_step(fdlbm_ctx *ctx, int64_t n_steps);

/* Check interval of fdlbm_step in steps (0, the default: no check, fully
 * asynchronous; 1: the exact step, at one synchronisation per step).
 * FDLBM_E_INVALID if negative. */
int fdlbm_set_sync_check(fdlbm_ctx *ctx, int64_t every);

/* Synchronise and report the stability record: *step = the first step
 * (counted like fdlbm_obs.step) in which a gas node had a non-finite or
 * negative density or temperature, or -1 if none did since the last
 * fdlbm_init_fields or fdlbm_load_state.  Batched steps keep each member's
 * record too.  FDLBM_E_STATE before fdlbm_init_fields. */
int fdlbm_last_step(fdlbm_ctx *ctx, int64_t *step);

/* Wait for the stream (no step of the method). */
int fdlbm_sync(fdlbm_ctx *ctx);

/* Synchronise and reduce the observables (FP64, deterministic order): the
 * per-species mass conserved up to the reacted mass (Eq.(37), summed over
 * gas and wall-emitted populations), the gas and solid energies and the
 * cumulative reaction heat (Eq.(42)) whose balance is Eq.(49)'s enthalpy
 * error, the Dirichlet-face heat, the body-force work, extrema and the
 * `bad` flag.  FDLBM_E_STATE before fdlbm_init_fields. */
int fdlbm_observe(fdlbm_ctx *ctx, fdlbm_obs *out);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): fdlbm_observe with the
 * same result, bitwise, that allocates nothing.  Its scratch -- the observe
 * kernel's per-block partial sums and their folded totals, at most
 * 1024 x (FDLBM_MAX_SPECIES + 9) + 64 doubles (139,776 bytes) -- lives in a
 * static device array of the library that each GPU holds until the process
 * ends; a context whose observables would not fit is rejected with
 * FDLBM_E_INVALID (none can with the library's fixed grid).  It calls no
 * allocating routine, host or device; the host side uses stack memory only.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (several host threads, or streams not ordered against each other) race.
 * Synchronises the context's stream. */
int fdlbm_observe_noalloc(fdlbm_ctx *ctx, fdlbm_obs *out);

/* Steady-state residual (the convergence test of the time-to-steady-state
 * measurement): for each field group q -- mole fractions X_j and temperature
 * and velocity at the gas nodes, solid temperature -- r_q = ||q(t) - q(s)||_2
 * / ((t - s) ||q(t)||_2) with s the step of the previous call, then a new
 * snapshot is taken.  r5[0..3] = X, T, u, T^s; r5[4] = their maximum.  The
 * first call after fdlbm_init_fields or fdlbm_load_state (no snapshot yet)
 * returns +inf.  Synchronises the stream.  FDLBM_E_STATE before the first
 * step. */
int fdlbm_residual(fdlbm_ctx *ctx, double *r5);

/* Copy a field into dst_host (double): n values, or Q*n for FDLBM_FIELD_POP.
 * RHO/U/T are the moments of the last step at gas nodes -- species density
 * and mixture velocity and temperature of Eq.(3), (5) with Eq.(25)'s
 * half-source terms (before the correction sources' energy) -- and the
 * wall state (rho_w of Eq.(39)-(41), U_w = 0, T_w) at wall nodes, 0
 * elsewhere; TS the solid temperature of Eq.(45)-(48); POP the stored
 * populations g of Eq.(23) (post-collision, the next step streams them);
 * WALL_R / WALL_DE the rate of Eq.(50) and the energy of the diffusive
 * exchange per wall node.  Valid after at least one step.  FDLBM_E_INVALID
 * for an unknown field or component. */
int fdlbm_get_field(fdlbm_ctx *ctx, int field, int comp, double *dst_host);

/* The same fields into a caller-owned device buffer dst_device (n doubles,
 * node order), without a host round trip: RHO, X, U, T, TS, KIND, WALL_R,
 * WALL_DE (not POP).  Enqueued on the context's stream (ordered after the
 * steps enqueued before it; no synchronisation); bitwise the values
 * fdlbm_get_field returns.  X_j = (rho_j / M_j) / sum_k (rho_k / M_k) at gas
 * and wall nodes, 0 elsewhere.  FDLBM_E_INVALID for POP, an unknown field or
 * component; FDLBM_E_STATE before the first step (TS and KIND: after
 * fdlbm_init_fields). */
int fdlbm_get_field_device(fdlbm_ctx *ctx, int field, int comp, double *dst_device);

/* Checkpoint (no step of the method): bytes needed, save to / restore from
 * a host buffer (bitwise: the whole device state of the step of
 * fdlbm_step, populations of Eq.(23), solid temperature, cumulative
 * counters of Eq.(42)/(49), step count).  host_buf is the caller's; load
 * requires a context with the same geometry and precision (else
 * FDLBM_E_INVALID) and resets the stability record. */
int fdlbm_state_bytes(const fdlbm_ctx *ctx, size_t *bytes);
int fdlbm_save_state(fdlbm_ctx *ctx, void *host_buf, size_t bytes);
int fdlbm_load_state(fdlbm_ctx *ctx, const void *host_buf, size_t bytes);

/* Concurrency within a step (default on): the wall and solid kernels run on
 * a second stream of the library's, beside the moments and collision kernels
 * on the context's stream, ordered by events; every step still completes on
 * the context's stream.  Off: all four on the context's stream, one after the
 * other (per-kernel timings then measure each kernel alone).  Results are
 * identical either way. */
int fdlbm_set_overlap(fdlbm_ctx *ctx, int enable);

/* Per-kernel timing with HIP events on the stream each kernel runs on.
 * While enabled (fdlbm_set_profiling(ctx, 1), which also resets the record),
 * each step brackets its kernels with events, for up to 4096 steps; fdlbm_kernel_times
 * synchronises and writes avg_ms[FDLBM_K_COUNT], the average duration in
 * milliseconds of each kernel group over the recorded steps (0 for a group
 * that did not run), and the number of recorded steps.  A group covers both
 * launches (periodic-wrap and plain) of its kernel. */
#define FDLBM_K_WALL 0     /* reactive wall                                  */
#define FDLBM_K_MOMENTS 1  /* streaming + moments + transport                */
#define FDLBM_K_COLLIDE 2  /* streaming + sources + collision + inlet/outlet */
#define FDLBM_K_SOLID 3    /* solid heat step                                */
#define FDLBM_K_COUNT 4
int fdlbm_set_profiling(fdlbm_ctx *ctx, int enable);
int fdlbm_kernel_times(fdlbm_ctx *ctx, double *avg_ms, int64_t *launches);

/* Node counts after fdlbm_set_geometry (Sec. 4.3: wall nodes are the
 * first solid nodes): gas (incl. inlet/outlet), wall, solid (incl. wall). */
int fdlbm_counts(const fdlbm_ctx *ctx, int64_t *n_gas, int64_t *n_wall, int64_t *n_solid);

/* ------------------------------------------------------------------------
 * Batches: many independent samples (contexts) advanced together.  Every
 * launch of a step serves all active samples at once: a persistent grid of
 * workgroups walks a device work list of (sample, block) pairs, so samples
 * of uneven size share the GPU without a launch per sample, and runs of
 * steps replay a captured HIP graph.  The physics of each sample is exactly
 * that of fdlbm_step on its own context (the same kernels per node and the
 * same per-block accumulation order, so the results are bitwise equal).
 * Members must be initialised, share lattice, species count, precision,
 * stream, wall position, solid-gas coupling, solid scheme and whether they
 * have several surface reactions, and keep their workspaces bound while the
 * batch lives (a member whose variant changes afterwards makes the next
 * fdlbm_batch_set_active fail).  Parameters
 * changed on a member after fdlbm_batch_bind_workspace take effect at the
 * next fdlbm_batch_set_active.  Each member's own calls (observe, residual,
 * get_field, save/load) keep working between batch steps; fdlbm_step on a
 * member while it is active in a batch is a call-order error the library
 * does not detect (the batch would then launch with the wrong parity).
 * ------------------------------------------------------------------------ */
typedef struct fdlbm_batch fdlbm_batch;

/* launch kinds of a batched step (persistent grids are set per kind) */
#define FDLBM_BL_WALL_FAST 0  /* wall nodes whose taps never wrap          */
#define FDLBM_BL_WALL_SLOW 1  /* wall nodes near a periodic face           */
#define FDLBM_BL_GAS_FAST 2   /* streaming + moments, no periodic wrap     */
#define FDLBM_BL_GAS_SLOW 3   /* streaming + moments near a periodic face  */
#define FDLBM_BL_COLLIDE 4    /* sources + collision + inlet/outlet        */
#define FDLBM_BL_SOLID 5      /* solid heat step                           */
#define FDLBM_BL_COUNT 6

/* Group n contexts (array copied; the contexts stay owned by the caller and
 * must outlive the batch).  All samples start active. */
int fdlbm_batch_create(fdlbm_ctx *const *ctxs, int n, fdlbm_batch **out);
void fdlbm_batch_destroy(fdlbm_batch *b);
const char *fdlbm_batch_last_error(const fdlbm_batch *b);

/* Caller-allocated device workspace (per-sample parameter and buffer tables,
 * work lists), >= fdlbm_batch_workspace_bytes, 256-byte aligned, kept alive
 * until destroy.  Binding uploads the tables (synchronises the stream). */
int fdlbm_batch_workspace_bytes(const fdlbm_batch *b, size_t *bytes);
int fdlbm_batch_bind_workspace(fdlbm_batch *b, void *dev_ptr, size_t bytes);

/* active[n]: nonzero = the sample advances in fdlbm_batch_step, zero = its
 * state is frozen (e.g. converged).  Re-uploads parameters and work lists;
 * synchronises the stream.  Captured graphs stay valid (the kernels read the
 * list lengths from device memory). */
int fdlbm_batch_set_active(fdlbm_batch *b, const uint8_t *active);

/* Advance every active sample by n_steps: whole runs of graph_steps steps
 * replay a captured graph (captured on first use per parity), the rest are
 * launched directly (all of them on the NULL stream, which cannot be
 * captured).  Asynchronous on the stream; updates the members' step
 * counters. */
int fdlbm_batch_step(fdlbm_batch *b, int64_t n_steps);

/* Stability check of a batch (failure detection of the step, as
 * fdlbm_step's checked mode): synchronises the stream and reads every
 * sample's stability record.  FDLBM_E_UNSTABLE if a sample has had a gas
 * node with a non-finite or negative density or temperature, with *sample
 * the lowest such sample index and *step its first such step (counted like
 * fdlbm_obs.step, the same as fdlbm_last_step on that member); otherwise
 * FDLBM_OK with both set to -1. */
int fdlbm_batch_check(fdlbm_batch *b, int *sample, int64_t *step);

/* Persistent grid per launch kind (FDLBM_BL_COUNT values, positive multiples
 * of 8 workgroups; NULL keeps them) and steps per captured graph (even, > 0;
 * 0 keeps it).  Drops captured graphs. */
int fdlbm_batch_set_grid(fdlbm_batch *b, const int *grid, int graph_steps);
int fdlbm_batch_get_grid(const fdlbm_batch *b, int *grid, int *graph_steps);

/* As fdlbm_set_overlap for the batched steps (default on): the wall and
 * solid launches run on a second stream beside the moments and collision
 * launches, inside the captured graphs too.  Drops captured graphs. */
int fdlbm_batch_set_overlap(fdlbm_batch *b, int enable);

/* Autotuner of the launch shapes: for each candidate grid (256 ... 16384
 * workgroups, capped at one workgroup per block of work), every launch kind
 * is timed with HIP events over `steps` steps after one warm-up step, and each
 * kind keeps its fastest grid (written to grid_out[FDLBM_BL_COUNT] if not
 * NULL).  The tuning steps are real steps of the active samples (their step
 * counters advance).  Synchronises the stream. */
int fdlbm_batch_autotune(fdlbm_batch *b, int steps, int *grid_out);

#ifdef __cplusplus
}
#endif
#endif
