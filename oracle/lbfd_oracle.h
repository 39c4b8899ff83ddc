/*
 * lbfd_oracle.h -- plain FP64 CPU oracle of the coupled low-Mach
 * lattice-Boltzmann / finite-difference / phase-field (LB-FD-PF) step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this library; only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the HIP implementation: every formula below is written out
 * again here from the paper (Namdar, Norouzi, Varnik, "A low-Mach phase
 * field-lattice Boltzmann-finite difference model for reactive gas flows
 * propagating through complex shaped particle assemblies").
 *
 * Units: lattice units (dx = dt = 1) except temperatures, in kelvin.
 * Layout of every field: x fastest, then y, then z (idx = (z*ny + y)*nx + x);
 * multi-component fields are stored component-major ([k][cell]).
 */
#ifndef LBFD_ORACLE_H
#define LBFD_ORACLE_H

#include <stdint.h>

#define ORC_MAXS 16 /* species */
#define ORC_MAXR 32 /* reactions */

/* LB boundary kinds per face (-x,+x,-y,+y,-z,+z) */
enum { ORC_LB_PERIODIC = 0, ORC_LB_WALL = 1, ORC_LB_INLET = 2, ORC_LB_OUTLET = 3,
       ORC_LB_CHAR_OUTLET = 4 };
/* FD boundary kinds per face */
enum { ORC_FD_PERIODIC = 0, ORC_FD_DIRICHLET = 1, ORC_FD_NEUMANN = 2 };
/* phase bits for orc_step */
enum { ORC_PH_LB = 1, ORC_PH_FD = 2, ORC_PH_CHEM = 4, ORC_PH_ALL = 7 };
/* readable fields */
enum { ORC_F_RHO = 0, ORC_F_U = 1, ORC_F_T = 2, ORC_F_Y = 3, ORC_F_PH = 4,
       ORC_F_POP = 5, ORC_F_DIVU = 6, ORC_F_OUTW = 7 /* ny*nz values */ };
/* diagnostics vector layout (doubles) */
enum { ORC_D_MASS = 0, ORC_D_SPECIES = 1, ORC_D_ENTHALPY = 17, ORC_D_KINETIC = 18,
       ORC_D_UMAX = 19, ORC_D_TMIN = 20, ORC_D_TMAX = 21, ORC_D_NONFINITE = 22,
       ORC_D_TAUBAD = 23, ORC_D_NEGY = 24, ORC_D_FLAGGED = 25, ORC_D_FALLBACK = 26,
       ORC_D_STEP = 27, ORC_D_LEN = 28 };

typedef struct {
    int32_t dim, nx, ny, nz;          /* dim 2 -> D2Q9 (nz must be 1), 3 -> D3Q19 */
    int32_t ns, nr;                   /* species, reactions                       */
    int32_t lb_bc[6];                 /* ORC_LB_*                                 */
    int32_t fd_bc[6];                 /* ORC_FD_*                                 */
    double  fd_val[6][1 + ORC_MAXS];  /* Dirichlet face values: T, then Y_k       */
    double  A_u, A_T, eta, T_s;       /* interface coupling, solid temperature    */
    double  Pr, cp, rho_in, T_in, nu_in, S_suth;
    int32_t mu_model;                 /* 0 constant viscosity, 1 Sutherland       */
    int32_t transport;                /* 0 single gas, 1 Wilke mixture rules      */
    double  u_in[3], F_b[3];          /* inlet velocity, body force               */
    double  Y_in[ORC_MAXS];           /* inlet composition (fixes reference M)    */
    double  Le[ORC_MAXS];             /* Lewis numbers                            */
    int32_t n_sub;                    /* explicit chemistry substeps per step     */
    double  theta_ign;                /* reaction-activity flag threshold [K]     */
    double  M[ORC_MAXS], dhf[ORC_MAXS], mu_star[ORC_MAXS];
    int32_t nu_f[ORC_MAXR][ORC_MAXS], nu_r[ORC_MAXR][ORC_MAXS];
    double  A[ORC_MAXR], beta[ORC_MAXR], theta[ORC_MAXR];
    int32_t rev[ORC_MAXR];
    double  lnKc_a[ORC_MAXR], lnKc_b[ORC_MAXR];
    /* closed domain (Sec. 3.1, the P0(t) of Eq. rho-in-terms-of-P0-and-T and
     * the dP0/dt term of Eq. energy-transport-DI-version): 0 keeps P0 fixed */
    int32_t closed;
    double  r_gas;                    /* R / M_ref in the units of cp            */
    double  p0;                       /* P0 / P0_in, kept by the oracle          */
    /* sharp-interface reference mode (Sec. 4: the phase-field coupling switched
     * off, bulk phases separated at phi = 1/2): cells with phi_s >= 1/2 are
     * solid -- halfway bounce-back for the populations, a ghost at T_s for
     * heat conduction, no species or advective flux -- and the drag and
     * heat-exchange terms vanish.  0: the diffuse-interface model */
    int32_t si;
    /* characteristic (non-reflecting) outlet, ORC_LB_CHAR_OUTLET on +x: the
     * relaxation factor sigma of the incoming wave amplitude, Sec. 4 open
     * boundary after Poinsot and Lele (> 0) */
    double  outlet_sigma;
    /* reaction step (Lie-split after transport; the paper takes its
     * integrator from its kinetics library):
     *   0  n_sub explicit Euler sub-steps,
     *   1  n_sub linearly implicit (Rosenbrock) Euler sub-steps with the
     *      analytic Jacobian of the rates at the sub-step's density,
     *   2  explicit Euler with a per-cell count n = min(n_sub, max(1,
     *      ceil(2 kappa))) of equal sub-steps, kappa the largest diagonal
     *      entry |d f_i / d y_i| of that Jacobian at the cell's state      */
    int32_t chem_scheme;
    /* species heat capacities c_p,k (Sec. 3.3, Eq. energy-transport-DI-
     * version): with cpk = 1 the mixture has c_p = sum_k Y_k c_p,k (in the
     * temperature equation, lambda = mu c_p/Pr, rho D_k = lambda/(c_p Le_k),
     * the reaction step and the enthalpy) and the temperature equation gets
     * the species heat-flux term -(sum_k c_p,k j_k) . grad T; cpk = 0: every
     * species at cp */
    int32_t cpk;
    double  cp_k[ORC_MAXS];
} orc_setup;

typedef struct orc_ctx orc_ctx;

orc_ctx* orc_create(const orc_setup* s, const double* phi_solid);
void     orc_destroy(orc_ctx* o);
/* T[N], Y[ns*N] (may be NULL when ns == 0), u[dim*N] (NULL -> at rest) */
int      orc_init_state(orc_ctx* o, const double* T, const double* Y, const double* u);
/* overwrite the post-stream populations (Q*N, natural layout) and, if not
 * NULL, the thermal divergence (N) -- restores a saved state */
int      orc_set_populations(orc_ctx* o, const double* g, const double* divu);
/* velocity inlet profile: u[a][z*ny + y] for a < dim (the inlet velocity of
 * each row of the -x face); NULL returns to the uniform u_in */
int      orc_set_inlet_profile(orc_ctx* o, const double* u);
int      orc_step(orc_ctx* o, int32_t n, int32_t phase_mask);
int      orc_read(const orc_ctx* o, int32_t field, int32_t comp, double* out);
void     orc_diag(const orc_ctx* o, double* out /* ORC_D_LEN */);
int32_t  orc_nthreads(void);
void     orc_set_threads(int32_t n);  /* OpenMP threads of the next steps (n > 0) */

/* unit hooks used by the pins */
void orc_eq_source(int32_t dim, double rho, const double* u, double Ph, const double* G,
                   const double* F, double divu, double* geq, double* xi);
void orc_lattice(int32_t dim, int32_t* c /* Q*3 */, double* w /* Q */);
void orc_mixture(const orc_setup* s, double T, const double* Y,
                 double* mu, double* lam, double* rhoD);
double orc_eos(const orc_setup* s, double T, const double* Y);
/* production rates omega_k and heat release omega_T (Eqs. 8 and 9) */
void orc_rates(const orc_setup* s, double T, const double* Y, double rho, double* wk,
               double* wT);
/* right-hand side of the reaction step at fixed density, f = (omega_k/rho,
 * omega_T/(rho cp)) (ns + 1 values), and its Jacobian J[i][m] = d f_i/d y_m
 * with y = (Y_1 .. Y_ns, T), row-major (ns + 1)^2 */
void orc_rates_jacobian(const orc_setup* s, double T, const double* Y, double rho, double* f,
                        double* J);
/* 0-D isobaric reactor: nsteps time steps of the reaction step each */
void orc_reactor(const orc_setup* s, double* T, double* Y, int32_t nsteps);
/* fd phase alone with u forced to zero (conservation pin); writes T*, Y* */
int  orc_fd_only(orc_ctx* o, double* Tstar, double* Ystar);
/* thermodynamic pressure ratio P0 / P0_in of the current state */
double orc_p0(const orc_ctx* o);

#endif
