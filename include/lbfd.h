/*
 * lbfd.h -- C ABI of the MI355X (gfx950) implementation of the coupled
 * low-Mach lattice-Boltzmann / finite-difference / phase-field (LB-FD-PF)
 * time step for reactive gas flow through a particle bed given as a diffuse
 * solid phase field (Namdar, Norouzi, Varnik, "A low-Mach phase field-lattice
 * Boltzmann-finite difference model for reactive gas flows propagating
 * through complex shaped particle assemblies").
 *
 * One call of lbfd_step advances every cell by one time step:
 *   1. LB collision and streaming of the pressure-based populations g_i
 *      (Sec. 3.3, Eqs. pop-g, body-force, eq-pop-f, eq-pop-g) with the
 *      interface drag F_drag = -A_u mu phi_f phi_s^2 u / eta^2
 *      (Sec. 3.2.1, Eq. Fdrag-empirical-law);
 *   2. FD advection-diffusion of T and Y_k (Sec. 3.2.2, Eq.
 *      volume-averaged-species-equation-5; Sec. 3.3, Eq.
 *      energy-transport-DI-version) with the interface heat exchange
 *      S_I = A_T lambda phi_f phi_s^2 (T_s - T)/eta^2 (Eq. diffusion-heat-flux-3);
 *   3. per-cell reaction sources omega_k, omega_T (Eqs. 8 and 9) from a plain
 *      Arrhenius mass-action table, integrated with n_sub explicit sub-steps;
 *   4. FP64 conservation diagnostics.
 * Closures: ideal-gas EOS at fixed thermodynamic pressure (Sec. 3.1),
 * Sutherland viscosity (Sec. 4, Eq. muT), lambda = mu cp/Pr (Eq. lambdaT),
 * Wilke mixture rules (Sec. 4.4, Eqs. muT_mix, phi_mix, conduct_mix).
 *
 * Units: lattice units (dx = dt = 1) except temperatures in kelvin.
 * Field layout everywhere: x fastest, then y, then z; multi-component fields
 * component-major.  Host I/O is FP64 whatever the device precision.
 * Lattices: D2Q9 (dim 2, nz = 1) or D3Q19 (dim 3).  Population order:
 * rest; +x,-x,+y,-y,+z,-z; then the diagonal pairs (c, -c):
 *   D2Q9:  (1,1),(-1,-1),(1,-1),(-1,1)
 *   D3Q19: (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),
 *          (-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1)
 *
 * Ownership: host arrays are read during the call and never retained.  The
 * device workspace and the HIP stream belong to the caller, must outlive the
 * context, and the library never allocates or frees device memory.
 * Errors: every call returns lbfd_status (0 = OK, negative = error) and no
 * C++ exception crosses the ABI; lbfd_last_error gives the message.  set_*
 * calls leave the context unchanged on error.  A context is bound to one
 * stream and is not thread-safe; distinct contexts are independent.
 */
#ifndef LBFD_H
#define LBFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBFD_MAX_SPECIES 16
#define LBFD_MAX_REACTIONS 32

typedef struct lbfd_ctx lbfd_ctx;

typedef enum {
    LBFD_OK = 0,
    LBFD_E_INVAL = -1,       /* bad argument or parameter out of the stable range */
    LBFD_E_NOMEM = -2,       /* workspace too small                              */
    LBFD_E_DEVICE = -3,      /* HIP runtime error                                */
    LBFD_E_STATE = -4,       /* call out of order (e.g. step before init_state)  */
    LBFD_E_NUMERIC = -5,     /* non-finite values appeared in a step             */
    LBFD_E_UNSUPPORTED = -6  /* valid request the library does not implement     */
} lbfd_status;

typedef enum { LBFD_FP64 = 0, LBFD_FP32 = 1 } lbfd_precision;

/* LB boundary kind per face (-x,+x,-y,+y,-z,+z).  The velocity inlet is
 * allowed on the -x face only and the pressure outlet on the +x face only. */
typedef enum {
    LBFD_LB_PERIODIC = 0,
    LBFD_LB_WALL = 1,             /* halfway bounce-back (no slip)                 */
    LBFD_LB_VELOCITY_INLET = 2,   /* equilibrium at (rho_in, u_in, local P_h)      */
    LBFD_LB_PRESSURE_OUTLET = 3,  /* equilibrium at (local rho, local u, P_h = 0)  */
    LBFD_LB_CHARACTERISTIC_OUTLET = 4 /* non-reflecting open outlet (the Poinsot-Lele
                                     characteristic treatment the paper uses, Sec. 4):
                                     equilibrium at (local rho, local u, P_out) with
                                     P_out = w + rho c_s u_x, where w, the amplitude
                                     of the wave entering through the face, is kept
                                     per outlet row and relaxed towards P_h = 0:
                                     w <- w - K P_h, K = outlet_sigma c_s (1 - Ma^2)/nx,
                                     Ma = |u_in|/c_s; w starts at 0 (init_state) */
} lbfd_lb_bc;

/* FD boundary kind per face; the +/- faces of an axis must both be periodic
 * or both non-periodic, and so must the LB kinds.  An FD-periodic face needs
 * an LB-periodic one; an LB-periodic face may instead carry an FD Dirichlet
 * temperature (a thermal wall across which the flow is periodic: plug flow
 * between isothermal walls), but no zero-gradient one. */
typedef enum {
    LBFD_FD_PERIODIC = 0,
    LBFD_FD_DIRICHLET = 1,       /* cell-centred ghost at the face value           */
    LBFD_FD_ZERO_GRADIENT = 2    /* ghost copies the boundary cell                 */
} lbfd_fd_bc;

typedef struct {
    int32_t dim, nx, ny, nz;     /* dim 2 -> D2Q9 (nz must be 1), dim 3 -> D3Q19   */
    int32_t precision;           /* lbfd_precision                                 */
    int32_t n_species;           /* 0 .. LBFD_MAX_SPECIES                          */
    int32_t lb_bc[6];            /* lbfd_lb_bc per face                            */
    int32_t fd_bc[6];            /* lbfd_fd_bc per face                            */
} lbfd_grid;

typedef struct {
    double A_u, A_T, eta, T_solid;   /* interface coupling (Eqs. Fdrag-empirical-law,
                                        diffusion-heat-flux-3), interface thickness
                                        in cells, solid temperature [K]             */
    double Pr, cp, rho_in, T_in, nu_in, sutherland_S;
    int32_t mu_model;                /* 0 constant viscosity, 1 Sutherland          */
    int32_t transport_model;         /* 0 single gas (lambda = mu cp/Pr),
                                        1 Wilke mixture rules with mu*_k            */
    double u_in[3], body_force[3];   /* inlet velocity, body force                  */
    double Y_in[LBFD_MAX_SPECIES];   /* inlet composition; fixes the reference molar
                                        mass of the EOS                             */
    double Le[LBFD_MAX_SPECIES];     /* Lewis numbers: rho D_k = lambda/(cp Le_k)   */
    double fd_face[6][1 + LBFD_MAX_SPECIES]; /* Dirichlet values per face: T, Y_k   */
    int32_t n_sub;                   /* explicit reaction sub-steps per step (>= 1) */
    double ign_threshold;            /* FP32 mode: a cell's reaction step runs in
                                        FP64 when |omega_T| dt/(rho cp) exceeds it [K] */
    int32_t closed;                  /* 1: closed domain (Sec. 3.1): the thermodynamic
                                        pressure P0(t) follows from the fixed mass,
                                        P0 / P0_in = sum(M/T at init) / sum(M/T), taken
                                        after every step; it scales the EOS, and its
                                        change over the previous step enters the
                                        temperature equation (Eq. energy-transport-
                                        DI-version) and the thermal divergence.  No
                                        inlet or outlet face.  init_state starts P0 at
                                        P0_in with the mass of the state it is given;
                                        a checkpoint restore also sets the P0 state
                                        (lbfd_set_p0_state).  0: P0 fixed             */
    double r_gas;                    /* closed domain: R / M_ref in the units of cp,
                                        0 <= r_gas < cp (the lagged dP0/dt term then
                                        settles with the ratio r_gas/cp < 1)         */
    double T_max;                    /* highest temperature the run is expected to
                                        reach [K] (e.g. the flame temperature); the
                                        stability rule (lbfd_stability) is evaluated
                                        up to the largest of T_max, T_in, T_solid, the
                                        Dirichlet face temperatures and, from
                                        lbfd_init_state on, the initial state's
                                        maximum.  0: no bound beyond those           */
    int32_t chem_scheme;             /* reaction step of one time step (after the
                                        transport, Lie splitting; Eqs. 8, 9):
                                        0: n_sub explicit Euler sub-steps;
                                        1: n_sub linearly implicit (one-stage
                                           Rosenbrock) Euler sub-steps with the
                                           analytic Jacobian of the rates at the
                                           sub-step's density: (I - h J) dy = h f
                                           (no reaction bound in the stability
                                           rule);
                                        2: per cell, n = min(n_sub, max(1,
                                           ceil(2 kappa))) explicit sub-steps,
                                           kappa = max_i |J_ii| at the cell.
                                        1 and 2 run in FP64 (in FP32 mode every
                                        cell's reaction step goes to the FP64
                                        island) and take at most 9 species.   */
    double outlet_sigma;             /* characteristic outlet: relaxation factor of
                                        the incoming wave (> 0; Poinsot and Lele
                                        suggest about 0.25); unused otherwise       */
    int32_t sharp_interface;         /* 1: sharp-interface reference mode (Sec. 4: the
                                        coupling to the phase field switched off, the
                                        bulk phases separated at phi = 1/2).  Cells
                                        with phi >= 1/2 are solid: they keep their
                                        state and populations and report u = 0,
                                        P_h = 0; a fluid cell bounces its populations
                                        back (halfway) at links to them and sees a
                                        solid neighbour as a ghost cell at T_solid
                                        with the fluid cell's own composition (in
                                        diffusion, convection and the density
                                        gradient); the drag and heat-exchange terms
                                        vanish.  Up to 4 species, exact reaction step
                                        only (no surrogate), no halo exchange.
                                        0: the diffuse-interface model               */
} lbfd_params;

typedef struct {
    int32_t n_species, n_reactions;
    const double* M;          /* [ns] molar masses                                */
    const double* dhf;        /* [ns] formation enthalpy per unit mass [cp*K]     */
    const double* mu_star;    /* [ns] species viscosity / reference viscosity     */
    const int32_t* nu_f;      /* [nr][ns] reactant stoichiometric coefficients,
                                 0..3, summing to at most 4 per reaction         */
    const int32_t* nu_r;      /* [nr][ns] product stoichiometric coefficients,
                                 0..3, summing to at most 4 per reaction         */
    const double* A;          /* [nr] k_f = A T^beta exp(-theta/T)                */
    const double* beta;       /* [nr]                                             */
    const double* theta;      /* [nr] activation temperature [K]                  */
    const int32_t* reversible;/* [nr] 0/1; k_r = k_f / exp(lnKc_a + lnKc_b/T)     */
    const double* lnKc_a;     /* [nr]                                             */
    const double* lnKc_b;     /* [nr]                                             */
    const double* cp;         /* [ns] species heat capacities c_p,k in the units of
                                 params.cp, or NULL (every species at params.cp).
                                 Given, the mixture has c_p = sum_k Y_k c_p,k (in
                                 the temperature equation, lambda = mu c_p/Pr,
                                 rho D_k = lambda/(c_p Le_k), the reaction step
                                 and the enthalpy) and the temperature equation
                                 gets the species heat-flux term
                                 -(sum_k c_p,k j_k) . grad T (Sec. 3.3, Eq.
                                 energy-transport-DI-version).  Single-gas
                                 transport, the explicit reaction scheme, no
                                 surrogate, no sharp-interface mode, at most 9
                                 species (LBFD_E_UNSUPPORTED otherwise)       */
} lbfd_mechanism;

typedef struct {
    double mass;                          /* sum rho                                 */
    double species_mass[LBFD_MAX_SPECIES];/* sum rho Y_k                             */
    double enthalpy;                      /* sum rho (cp T + sum_k dhf_k Y_k)        */
    double kinetic;                       /* sum rho |u|^2/2 of the last LB step     */
    double umax, Tmin, Tmax;
    int64_t n_nonfinite, n_tau_bad, n_negY, n_flagged_fp64, n_fallback, step;
    int64_t n_fallback_reason[4];         /* surrogate cell-steps failing each check:
                                             envelope, overdraw, residual, positivity
                                             (a cell may fail several)               */
    double p0_ratio;                      /* P0 / P0_in for the next step (1 unless
                                             the domain is closed)                   */
} lbfd_diag;

typedef enum {
    LBFD_F_RHO = 0,          /* EOS of the current state                          */
    LBFD_F_U = 1,            /* component 0..dim-1; moments of the current populations */
    LBFD_F_T = 2,
    LBFD_F_Y = 3,            /* component 0..ns-1                                 */
    LBFD_F_PH = 4,           /* hydrodynamic pressure of the current populations  */
    LBFD_F_POPULATIONS = 5,  /* component 0..Q-1, post-stream, natural layout     */
    LBFD_F_DIVU = 6,         /* thermal velocity divergence used by the next step */
    LBFD_F_OUTLET_WAVE = 7   /* characteristic outlet: the incoming wave amplitude w
                                per outlet row, ny*nz values (z*ny + y); part of a
                                checkpoint (lbfd_set_outlet_wave restores it)    */
} lbfd_field;

/* phase bits of lbfd_step_phase (test hook; lbfd_step runs all three) */
enum { LBFD_PHASE_LB = 1, LBFD_PHASE_FD = 2, LBFD_PHASE_CHEM = 4, LBFD_PHASE_ALL = 7 };

/* ------------------------------------------------------------------------
 * Explicit-stability rule (host only, no device needed).  The FD transport is
 * one forward-Euler step with first-order upwind convection, conservative
 * central diffusion and the interface heat exchange (Sec. 3.3); the reaction
 * step is n_sub explicit sub-steps of Eqs. 8 and 9.  Per cell the FD update is
 * a convex combination of the old values (hence bounded, non-oscillating)
 * when its diagonal weight 1 - (sum_faces lambda_f/(rho cp) + H/(rho cp) +
 * sum_a |u_a|) stays positive.  Over the temperature range [T_lo, T_hi]:
 *   tau_lo   = mu/(rho cs^2) + 1/2 at T_lo (viscosity and density grow and
 *              fall with T), must exceed 0.501;
 *   alpha_hi = lambda/(rho cp), D_hi = max_k lambda/(rho cp Le_k) at T_hi,
 *              with the closure of the params (single gas, or the Wilke
 *              mixture at the inlet composition) and rho of the inlet mixture;
 *   h_hi     = A_T alpha_hi max(phi_f phi_s^2)/eta^2, the maximum 4/27 at
 *              phi_s = 2/3;
 *   u_sum    = sqrt(dim) 0.1, the low-Mach limit |u| <= 0.1;
 *   fd_sum   = 2 dim max(alpha_hi, D_hi) + h_hi + u_sum, must be <= 0.9;
 *   kappa_hi = max_k of species k's pseudo-first-order consumption rate,
 *              sum_j nu_kj k_j prod_m [X_m]^(nu_mj - delta_mk) over the
 *              forward and (reversible) reverse sides, at T_hi with
 *              [X_m] = rho max(Y_in,m, 0.01)/M_m (every species counted at
 *              one per cent at least, so that products absent at the inlet
 *              still count);
 *   h_kappa  = kappa_hi / n_sub, must be <= 0.5.
 * lbfd_set_params, lbfd_set_mechanism and lbfd_init_state apply this rule and
 * return LBFD_E_INVAL (message naming the failed bound) when it fails.
 * ------------------------------------------------------------------------ */
typedef struct {
    double T_lo, T_hi;   /* temperature range the bounds were evaluated over [K]  */
    double tau_lo;       /* relaxation time at T_lo                               */
    double alpha_hi, D_hi, h_hi, u_sum;
    double fd_sum;       /* must be <= 0.9                                        */
    double kappa_hi;     /* 0 without a mechanism                                 */
    double h_kappa;      /* must be <= 0.5                                        */
    int32_t violated;    /* bits: 1 tau_lo, 2 fd_sum, 4 h_kappa, 8 a non-finite
                            rate or property                                      */
} lbfd_stability_report;

/* The explicit steps of Sec. 3.3 (forward Euler FD update, n_sub explicit
 * reaction sub-steps) and the BGK relaxation of Sec. 3.3 are stable under
 * the bounds of this rule.
 * Evaluate the rule for a grid, params and mechanism (mech may be NULL: no
 * reaction bound, and a Wilke closure then needs it and is skipped) over the
 * temperatures T_in, T_solid, the Dirichlet faces, params->T_max and the
 * extra range [T_lo, T_hi] (pass 0, 0 for none).  Fills *out (may be NULL);
 * LBFD_OK when every bound holds, LBFD_E_INVAL otherwise or for bad
 * arguments. */
lbfd_status lbfd_stability(const lbfd_grid* grid, const lbfd_params* params,
                           const lbfd_mechanism* mech, double T_lo, double T_hi,
                           lbfd_stability_report* out);

/* Bytes of device workspace a grid needs (256-byte aligned base expected).
 * The grid is the paper's Cartesian domain of volume elements (Sec. 2, the
 * averaging cells of Eq. def-volume-average; lattice units, one cell per
 * element).  LBFD_E_INVAL for a grid the library cannot hold (see
 * lbfd_grid; at most 2^31 / Q cells, 32-bit plane offsets). */
lbfd_status lbfd_workspace_bytes(const lbfd_grid* grid, size_t* bytes);

/* Create a context for one grid (Sec. 2, Eq. def-volume-average: the cells
 * over which every field is averaged) on the current HIP device.
 * dev_workspace: caller-owned device buffer of at least lbfd_workspace_bytes,
 * 256-byte aligned (LBFD_E_INVAL otherwise, LBFD_E_NOMEM when too small);
 * hip_stream: hipStream_t (or NULL for the null stream) on which every kernel
 * of this context runs.  *out receives the context (host memory owned by the
 * library until lbfd_destroy); LBFD_E_DEVICE when no device is current. */
lbfd_status lbfd_create(const lbfd_grid* grid, void* dev_workspace, size_t bytes,
                        void* hip_stream, lbfd_ctx** out);

/* Static solid phase field phi_s in [0, 1] (host, nx*ny*nz doubles, x
 * fastest): the volume fraction of the solid phase in each cell (Sec. 2, Eq.
 * phase-field-definition), e.g. from the diffuse profile of Eq. def-phi; the
 * fluid fraction is 1 - phi_s.  LBFD_E_INVAL for values outside [0, 1]. */
lbfd_status lbfd_set_phase_field(lbfd_ctx* ctx, const double* phi_solid);

/* Reaction mechanism of the sources omega_k = M_k sum_j s_kj Q_j (Sec. 3.2.2,
 * Eq. 8) and the heat release omega_T = -sum_k dh_f,k omega_k (Sec. 3.3,
 * Eq. 9), with mass-action rates of progress and Arrhenius rate constants;
 * M_k also enters the EOS (Eq. rho-in-terms-of-P0-and-T) and the Wilke rules
 * (Sec. 4.4, Eqs. muT_mix, phi_mix, conduct_mix).  Host tables, copied
 * during the call.  n_species must equal the grid's.  LBFD_E_INVAL for bad
 * tables, orders beyond the limits in lbfd_mechanism, or a mechanism that
 * breaks the stability rule with the params already set. */
lbfd_status lbfd_set_mechanism(lbfd_ctx* ctx, const lbfd_mechanism* mech);

/* Physical and coupling parameters (host struct, copied): the interface drag
 * coefficient A_u and thickness eta (Sec. 3.2.1, Eq. Fdrag-empirical-law), the
 * heat-exchange coefficient A_T and solid temperature (Sec. 3.3, Eq.
 * diffusion-heat-flux-3), Sutherland viscosity and conductivity (Sec. 4, Eqs.
 * muT and lambdaT), the inlet state fixing the EOS reference (Sec. 3.1, Eq.
 * rho-in-terms-of-P0-and-T) and the boundary values.  LBFD_E_INVAL for
 * non-physical values (eta, cp, Pr, rho_in, T_in, nu_in, T_solid <= 0,
 * |u_in| > 0.1, n_sub outside 1..4096, inlet fractions not summing to 1) and
 * for parameters breaking the stability rule (lbfd_stability); the context
 * is then unchanged.  May be called between steps. */
lbfd_status lbfd_set_params(lbfd_ctx* ctx, const lbfd_params* params);

/* Initial state (host FP64, x fastest): T[N], Y[ns*N] (NULL iff ns == 0),
 * u[dim*N] or NULL (rest).  Sets rho from the EOS (Sec. 3.1, Eq.
 * rho-in-terms-of-P0-and-T), divu = 0, P_h = 0 and the populations to the
 * equilibrium of Eqs. eq-pop-f and eq-pop-g; clears the diagnostics.  Needs
 * phase field, params and (ns > 0) mechanism first (LBFD_E_STATE).
 * LBFD_E_INVAL for non-positive or non-finite T, or for a state whose
 * temperatures break the stability rule (the previous state then stays). */
lbfd_status lbfd_init_state(lbfd_ctx* ctx, const double* T, const double* Y, const double* u);

/* Overwrite the post-stream populations g_i of Eq. pop-g (Q*N doubles,
 * natural layout, direction-major) and the thermal divergence of the source
 * term of Eq. body-force (N doubles, may be NULL); together with
 * lbfd_init_state this restores a checkpoint written with lbfd_read.
 * LBFD_E_INVAL for non-finite values; LBFD_E_STATE before lbfd_init_state. */
lbfd_status lbfd_set_populations(lbfd_ctx* ctx, const double* g, const double* divu);

/* Velocity inlet profile (Sec. 4.2 imposes a fully developed parabolic inflow):
 * u[a][z*ny + y] for a < dim, host memory, copied; the inlet row (y, z) of the
 * -x face then takes the equilibrium at (rho_in, u(y, z), local P_h) instead
 * of the uniform u_in of the params.  NULL returns to the uniform inlet.
 * LBFD_E_INVAL when the -x face is no velocity inlet, for non-finite values
 * or for |u| > 0.1 (the low-Mach limit). */
lbfd_status lbfd_set_inlet_profile(lbfd_ctx* ctx, const double* u);

/* Characteristic (non-reflecting) outlet of Sec. 4.1, after Poinsot and
 * Lele: overwrite the incoming wave amplitude w of every
 * outlet row (ny*nz doubles, z*ny + y, host memory) -- with lbfd_init_state
 * and lbfd_set_populations this restores a checkpoint.  LBFD_E_INVAL for
 * non-finite values or a grid without that outlet; LBFD_E_STATE before
 * lbfd_init_state. */
lbfd_status lbfd_set_outlet_wave(lbfd_ctx* ctx, const double* w);

/* Closed domain (Sec. 3.1): the thermodynamic-pressure state that a checkpoint
 * needs besides the fields: out/in[3] = {S0, p, p_prev}, the sum of M/T over
 * the cells of the initial state, P0/P0_in for the next step and for the last
 * one (host arrays of 3 doubles).  lbfd_set_p0_state, after lbfd_init_state,
 * restores it and rewrites the parameter blocks' EOS and dP0/dt terms.
 * LBFD_E_STATE when the domain is not closed or no state is set; LBFD_E_INVAL
 * for non-positive or non-finite values. */
lbfd_status lbfd_get_p0_state(lbfd_ctx* ctx, double* out);
lbfd_status lbfd_set_p0_state(lbfd_ctx* ctx, const double* in);

/* Enqueue n coupled steps on the context's stream (LB, then FD transport,
 * then reactions, as listed at the top of this file: Sec. 3.3 and Eqs. 8, 9);
 * returns without waiting.  LBFD_E_STATE before lbfd_init_state. */
lbfd_status lbfd_step(lbfd_ctx* ctx, int32_t n);

/* Enqueue n steps running only the phases in phase_mask (test hook): LB
 * (Sec. 3.3, the populations and the coupling force of Sec. 3.2.1), FD (the
 * transport of T and Y_k, Sec. 3.3) and CHEM (the sources of Eqs. 8 and 9).  Without
 * LB the velocity is zero and populations are untouched; without FD, T and Y
 * enter the reaction step unchanged; without CHEM no reaction is applied. */
lbfd_status lbfd_step_phase(lbfd_ctx* ctx, int32_t n, int32_t phase_mask);

/* Copy one field component to host (x fastest, N doubles; waits for the
 * stream): the low-Mach state of Sec. 3.1 -- rho (EOS of the current T, Y_k),
 * u and the hydrodynamic pressure P_h (moments of the current populations,
 * Eqs. eq-pop-f, eq-pop-g), T, Y_k -- the populations, or the thermal
 * divergence.  LBFD_E_INVAL for an unknown field or component. */
lbfd_status lbfd_read(lbfd_ctx* ctx, int32_t field, int32_t component, double* host_out);

/* Conservation sums of the state after the last step, FP64 (the integrals
 * of mass, species mass and enthalpy of the conservation laws of Sec. 3.1,
 * Eqs. mass-cons, species-cons, energy-cons, over the cells), and cumulative
 * counters (waits for the stream); returns LBFD_E_NUMERIC if n_nonfinite >
 * 0, with *out filled. */
lbfd_status lbfd_diagnostics(lbfd_ctx* ctx, lbfd_diag* out);

/* Wait for the context's stream (host synchronisation; no passage). */
lbfd_status lbfd_synchronize(lbfd_ctx* ctx);

/* Algorithmic HBM bytes one cell moves in one lbfd_step on this grid: each
 * array the fused step kernel reads or writes, once (populations in place,
 * T and Y_k read and written, divergence read and written, phi read). */
lbfd_status lbfd_step_bytes_per_cell(const lbfd_ctx* ctx, double* bytes);

/* ------------------------------------------------------------------------
 * Chemistry surrogate (FP32 mode).  A perceptron n_in -> 256 -> 256 -> n_out
 * with ReLU (BF16 operands on the matrix cores, FP32 accumulation and
 * biases) replaces the reaction sub-steps of every step (Eqs. 8 and 9): from
 * the post-transport state x = (T*, p, Y*_1..Y*_ns), n_in = 2 + ns,
 * n_out = ns, it predicts the step-integrated sources
 * w_k = rho* (Y_k^chem - Y*_k)/dt, de-standardised as mu_y + sd_y * yhat.
 * The prediction is projected to sum_k w_k = 0 (w_k -= Y*_k sum_m w_m) and
 * applied as Y_k = Y*_k + w_k/rho*, T = T* + w_T/(rho* c_p),
 * w_T = -sum_k dh_k w_k.  Before the projection a source that would take
 * more of a species than the cell holds (w_k < -rho* Y*_k) is clipped to
 * -rho* Y*_k.  A cell takes the exact FP64 reaction step instead (counted in
 * n_fallback and n_flagged_fp64) when an input lies outside the training
 * envelope widened on each side by 1 % of its range plus 0.05 sd_x, when
 * such a clip
 * exceeds 0.05 sd_y[k], when
 * |sum w| > 0.05 (sum |w| + sum_k sd_y[k]) before the projection, or when
 * the update would give some Y_k < -1e-8.
 * ------------------------------------------------------------------------ */

/* Install (or, with weights == NULL, remove) the surrogate.  Host arrays,
 * copied during the call:
 *   weights  FP32, row-major, concatenated: W1 [256][n_in], b1 [256],
 *            W2 [256][256], b2 [256], W3 [n_out][256], b3 [n_out];
 *   norm     mu_x [n_in], sd_x [n_in], mu_y [n_out], sd_y [n_out] (sd > 0);
 *   envelope lo [n_in], hi [n_in] of the training inputs (hi >= lo).
 * The feature p is the constant 1.  LBFD_E_UNSUPPORTED in FP64 mode or
 * outside 1 <= n_species <= 14; LBFD_E_INVAL on non-finite weights. */
lbfd_status lbfd_set_surrogate(lbfd_ctx* ctx, const float* weights, const float* norm,
                               const float* envelope);

/* Evaluate the installed surrogate on n states (device arrays, enqueued on
 * the context's stream): T [n], Y [n_species][n] in; raw (de-standardised
 * prediction after the overdraw clip, before projection) [n_species][n],
 * omega (after projection) [n_species][n] and fallback [n] out: 0 when the
 * update stands, else the failed checks, 1 envelope | 2 overdraw |
 * 4 residual | 8 positivity. */
lbfd_status lbfd_surrogate_eval(lbfd_ctx* ctx, const float* T, const float* Y, int32_t n,
                                float* raw, float* omega, int32_t* fallback);

/* Training pairs from the current state (device arrays, enqueued): for each
 * cell index cells[i] (linear, x fastest), x[i] = (T, 1, Y_1..Y_ns) as
 * [n][2 + ns] and the exact step-integrated source of one step of n_sub FP64
 * sub-steps, y[i] = rho (Y^chem - Y)/dt as [n][ns].  Indices outside the
 * grid give rows of NaN.  FP32 mode with a mechanism only. */
lbfd_status lbfd_sample_states(lbfd_ctx* ctx, const int32_t* cells, int32_t n, float* x,
                               float* y);

/* ------------------------------------------------------------------------
 * Surrogate training (offline, once per mechanism).  Mini-batch Adam
 * (Kingma and Ba) on the mean-square error of the standardised outputs,
 * L = mean over batch and outputs of (yhat - (y - mu_y)/sd_y)^2, with FP32
 * master weights and moments and bf16 matrix-core products (FP32
 * accumulation).  Deterministic: fixed-order reductions throughout.
 * The trainer owns no memory: the caller passes a device workspace of
 * lbfd_trainer_workspace_bytes(cfg) bytes, 256-byte aligned, and a stream;
 * data arrays (x [n][2 + ns], y [n][ns] as written by lbfd_sample_states,
 * batch indices [batch]) are device arrays that must stay valid while the
 * enqueued work runs.
 * ------------------------------------------------------------------------ */
typedef struct lbfd_trainer lbfd_trainer;
typedef struct {
    int32_t n_species;   /* 1..14: n_in = 2 + ns inputs, ns outputs */
    int32_t batch;       /* samples per step, a multiple of 256 */
    float beta1, beta2, eps;  /* Adam constants (e.g. 0.9, 0.999, 1e-8) */
} lbfd_train_cfg;

lbfd_status lbfd_trainer_workspace_bytes(const lbfd_train_cfg* cfg, size_t* bytes);
lbfd_status lbfd_trainer_create(const lbfd_train_cfg* cfg, void* dev_workspace, size_t bytes,
                                void* hip_stream, lbfd_trainer** out);
/* Standardisation statistics (FP64 mean and population standard deviation,
 * floored at 1e-12 max(|mu|, 1) and, for the mass-fraction inputs, at 1e-4)
 * and the input envelope [min, max] of n samples (enqueued). */
lbfd_status lbfd_trainer_fit_norm(lbfd_trainer* tr, const float* x, const float* y, int32_t n);
/* Master weights from the host (layout of lbfd_set_surrogate); resets the
 * Adam moments and step count (waits for the stream). */
lbfd_status lbfd_trainer_set_weights(lbfd_trainer* tr, const float* weights);
/* One Adam step with learning rate lr on the batch rows idx[0..batch) of the
 * n samples (indices outside [0, n) read as zero rows).  If loss is not NULL
 * it waits and returns the batch's loss before the update. */
lbfd_status lbfd_trainer_step(lbfd_trainer* tr, const float* x, const float* y, int32_t n,
                              const int32_t* idx, float lr, double* loss);
/* Gradient of the batch loss (host, weights layout) and the loss, without an
 * update (waits). */
lbfd_status lbfd_trainer_gradient(lbfd_trainer* tr, const float* x, const float* y, int32_t n,
                                  const int32_t* idx, float* grad, double* loss);
/* Weights, norm and envelope to the host in lbfd_set_surrogate's layouts
 * (any may be NULL; waits). */
lbfd_status lbfd_trainer_export(lbfd_trainer* tr, float* weights, float* norm, float* envelope);
lbfd_status lbfd_trainer_destroy(lbfd_trainer* tr);

/* The statistics of lbfd_trainer_fit_norm followed by lbfd_trainer_export's
 * norm and envelope, without a trainer, a workspace or any allocation: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  x [n][2 + n_species] and
 * y [n][n_species] are device arrays as written by lbfd_sample_states; norm
 * (2 (2 + ns) + 2 ns floats) and envelope (2 (2 + ns) floats) are host
 * arrays in lbfd_set_surrogate's layouts (either may be NULL, not both);
 * hip_stream as in lbfd_create.  The kernel stages the statistics in a
 * 4 KiB device array of the library (one per GPU, held until the process
 * ends), which bounds n_species to 1..14 (LBFD_E_UNSUPPORTED beyond);
 * LBFD_E_INVAL for n < 2 or null data.  Waits for the stream.  Calls on one
 * GPU share that array: calls that overlap on one GPU (other threads or
 * streams) race and must be serialised by the caller. */
lbfd_status lbfd_fit_norm_noalloc(int32_t n_species, const float* x, const float* y, int32_t n,
                                  float* norm, float* envelope, void* hip_stream);
const char* lbfd_trainer_last_error(const lbfd_trainer* tr);

/* ------------------------------------------------------------------------
 * Halo planes: the strided copies that a decomposition of the grid into slabs
 * along x exchanges between neighbouring slabs after every step (the one-cell
 * stencils of the LB streaming, Eq. pop-g, and of the FD transport, Eqs.
 * volume-averaged-species-equation-5 and energy-transport-DI-version, reach
 * one plane across a slab face).  A slab context holds its own planes
 * x = 1 .. nx - 2 and one halo plane on each side (x = 0 copies the left
 * neighbour's last own plane, x = nx - 1 the right neighbour's first); its x
 * faces are periodic.  After every lbfd_step(ctx, 1) each slab packs both
 * faces (face -1: towards its left neighbour, +1: towards its right one) and
 * then unpacks, on each face, the buffer its neighbour packed for it; the
 * own planes then evolve bitwise as in the undivided grid.  What travels
 * follows the AA parity of the state: T and Y_k of the own boundary plane
 * (as stored: T - T_solid in FP32 mode, so neighbours need equal T_solid)
 * and 5 population planes (3 in D2Q9; as stored: 36 g_i in FP32 mode) --
 * after an even
 * step the own boundary
 * plane's slots with c_x = -face, which become the neighbour's halo slots;
 * after an odd step the halo plane's slots with c_x = face, the populations
 * the step pushed across the face, which become the neighbour's own slots.
 * Buffer: plane after plane, [z][y] within a plane, populations then T then
 * Y_1..Y_ns, in the device precision: lbfd_halo_bytes bytes.  dev_buf:
 * caller-owned device memory; enqueued on the context's stream; LBFD_E_INVAL
 * for a face other than -1 / +1 or nx < 3; LBFD_E_STATE before init_state.
 * ------------------------------------------------------------------------ */
lbfd_status lbfd_halo_bytes(const lbfd_ctx* ctx, size_t* bytes);
lbfd_status lbfd_halo_pack(lbfd_ctx* ctx, int32_t face, void* dev_buf);
lbfd_status lbfd_halo_unpack(lbfd_ctx* ctx, int32_t face, const void* dev_buf);

/* Per-kernel launch timing (measurement hook).  While enabled, every launch
 * of the fused step kernel, of the FP64 reaction-island kernel and of the
 * surrogate kernel is bracketed by a pair of HIP events recorded on the
 * context's stream.
 * lbfd_kernel_time waits for the stream, returns the number of timed launches
 * of `kernel` (LBFD_KERNEL_*) since timing was enabled and their mean
 * duration in milliseconds (0 when there were none), and keeps counting.
 * Enabling restarts the count.  The events are created by the library on
 * first use and released by lbfd_destroy. */
enum { LBFD_KERNEL_STEP = 0, LBFD_KERNEL_ISLAND = 1, LBFD_KERNEL_SURROGATE = 2 };
lbfd_status lbfd_set_timing(lbfd_ctx* ctx, int32_t enable);
lbfd_status lbfd_kernel_time(lbfd_ctx* ctx, int32_t kernel, int64_t* launches, double* mean_ms);

lbfd_status lbfd_destroy(lbfd_ctx* ctx);
const char* lbfd_last_error(const lbfd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
