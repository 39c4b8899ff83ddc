/*
 * lbfd_oracle.c -- plain FP64 CPU oracle of the coupled LB-FD-PF step.
 *
 * TEST INFRASTRUCTURE ONLY (see lbfd_oracle.h).  Slow and obvious on purpose:
 * two population arrays with pull streaming, one phase after the other
 * (LB collide -> stream -> FD transport -> chemistry -> reductions), every
 * cell independently, FP64 throughout.
 *
 * Paper references are to sections and equations of the paper:
 *   Sec. 3.1   low-Mach system, ideal-gas EOS (Eq. rho-in-terms-of-P0-and-T)
 *   Sec. 3.2.1 interface drag (Eq. Fdrag-empirical-law)
 *   Sec. 3.2.2 species equation (Eq. volume-averaged-species-equation-5),
 *              production rates (Eq. 8)
 *   Sec. 3.3   interface heat exchange (Eq. diffusion-heat-flux-3),
 *              temperature equation (Eq. energy-transport-DI-version),
 *              heat release (Eq. 9), low-Mach LB (Eqs. pop-g, body-force,
 *              eq-pop-f, eq-pop-g), FD discretisation (upwind convection,
 *              central diffusion, explicit Euler)
 *   Sec. 4     Sutherland law (Eq. muT), conductivity (Eq. lambdaT)
 *   Sec. 4.4   mixture rules (Eqs. muT_mix, phi_mix, conduct_mix)
 * Readings of points the paper leaves open are stated where they are used.
 */
#include "lbfd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- lattice */
/* D2Q9 and D3Q19 (the paper only says "conventional" populations; the
 * lattices are fixed by the workloads).  Direction order is part of the
 * population read/write interface: rest, then axis pairs (+x,-x,+y,-y,+z,-z),
 * then diagonal pairs, each pair being (c, -c).                              */
static const int C2[9][3] = {{0, 0, 0},  {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                             {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const double W2[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int C3[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double CS2 = 1.0 / 3.0; /* lattice speed of sound squared */

struct orc_ctx {
    orc_setup s;
    int Q;
    long N;
    const int (*c)[3];
    const double* w;
    int opp[19];
    double Mbar_in;
    double Phi[ORC_MAXS][ORC_MAXS]; /* Wilke interaction matrix (constant: shared S) */
    int corr;                       /* species correction flux needed (unequal Le) */
    double *phi, *g, *gs, *T, *Y, *divu;
    double *u, *Ph, *rho_n, *Tst, *Yst, *qT;
    double* uprof;                  /* inlet velocity per row [3][ny*nz], or NULL */
    double* wout;                   /* characteristic outlet: incoming wave amplitude
                                       per row [ny*nz]                            */
    double diag[ORC_D_LEN];
    double p_prev, S0;               /* closed domain: previous P0 / P0_in, and the
                                        sum of M / T of the initial state        */
};

static long cidx(const orc_ctx* o, int x, int y, int z) {
    return ((long)z * o->s.ny + y) * o->s.nx + x;
}

/* Sharp-interface reference mode (Sec. 4): the bulk phases are separated at
 * phi = 1/2, so a cell with phi_s >= 1/2 is solid. */
static int is_solid(const orc_ctx* o, long id) { return o->s.si && o->phi[id] >= 0.5; }

/* The in-domain cell (x, y, z) after periodic wrapping is solid (0 when it
 * lies beyond a non-periodic face). */
static int solid_at(const orc_ctx* o, int x, int y, int z) {
    const orc_setup* s = &o->s;
    if (!s->si) return 0;
    int p[3] = {x, y, z}, n[3] = {s->nx, s->ny, s->nz};
    for (int a = 0; a < 3; ++a) {
        if (p[a] >= 0 && p[a] < n[a]) continue;
        if (s->fd_bc[2 * a + (p[a] < 0 ? 0 : 1)] != ORC_FD_PERIODIC) return 0;
        p[a] = (p[a] + n[a]) % n[a];
    }
    return is_solid(o, cidx(o, p[0], p[1], p[2]));
}

/* ---------------------------------------------------------------- closures */

/* Ideal-gas EOS at constant thermodynamic pressure (Sec. 3.1, Eq.
 * rho-in-terms-of-P0-and-T): rho = M P0/(R T).  Open domains keep P0 fixed,
 * so rho = rho_in (T_in/T)(M/M_in) with 1/M = sum_k Y_k/M_k.                 */
static double inv_mbar(const orc_setup* s, const double* Y) {
    double r = 0.0;
    for (int k = 0; k < s->ns; ++k) r += Y[k] / s->M[k];
    return r;
}
double orc_eos(const orc_setup* s, double T, const double* Y) {
    /* a closed domain scales the density with P0(t) / P0_in */
    const double p = s->closed ? s->p0 : 1.0;
    if (s->ns == 0) return p * (s->rho_in * (s->T_in / T));
    double mbar = 1.0 / inv_mbar(s, Y);
    double mbar_in = 1.0 / inv_mbar(s, s->Y_in);
    return p * (s->rho_in * (s->T_in / T) * (mbar / mbar_in));
}

/* Closed domain (Sec. 3.1): the mass m = int rho dV is fixed and the EOS makes
 * rho proportional to P0 M / T, so P0 = m R / int (M / T) dV.  With m taken
 * from the initial state at P0_in, the ratio is p = S0 / S, S = sum over the
 * cells of M / T (every cell of the diffuse-interface domain).  The sum is
 * compensated (Neumaier's variant of Kahan summation): dP0/dt is the
 * difference of two such sums, so their rounding must not depend on the order
 * in which the cells are added.                                            */
static double closed_sum(const orc_ctx* o) {
    const orc_setup* s = &o->s;
    double S = 0.0, c = 0.0;
    for (long id = 0; id < o->N; ++id) {
        double Y[ORC_MAXS];
        for (int k = 0; k < s->ns; ++k) Y[k] = o->Y[(long)k * o->N + id];
        const double mbar = s->ns ? 1.0 / inv_mbar(s, Y) : 1.0;
        const double x = mbar / o->T[id], t = S + x;
        c += fabs(S) >= fabs(x) ? (S - t) + x : (x - t) + S;
        S = t;
    }
    return S + c;
}

/* Sutherland law (Sec. 4, Eq. muT) written as a ratio to the inlet state so
 * that the reference temperature cancels: mu(T)/mu(T_in).                   */
/* Mixture heat capacity, c_p = sum_k Y_k c_p,k (cp when the species share it). */
static double cp_of(const orc_setup* s, const double* Y) {
    if (!s->cpk) return s->cp;
    double c = 0.0;
    for (int k = 0; k < s->ns; ++k) c += Y[k] * s->cp_k[k];
    return c;
}

static double sutherland_ratio(const orc_setup* s, double T) {
    if (s->mu_model == 0) return 1.0;
    double x = T / s->T_in;
    return x * sqrt(x) * (s->T_in + s->S_suth) / (T + s->S_suth);
}

/* Wilke interaction coefficient (Sec. 4.4, Eq. phi_mix). */
static double wilke_phi(double mu_k, double mu_j, double M_k, double M_j) {
    double a = 1.0 + sqrt((mu_k / mu_j) * sqrt(M_j / M_k));
    return a * a / (sqrt(8.0) * sqrt(1.0 + M_k / M_j));
}

/* Transport properties of one state.
 * single gas: mu from Sutherland, lambda = mu c_p/Pr (Eq. lambdaT) with the
 *             mixture c_p.
 * mixture:    mu_k = mu*_k mu_ref s(T), lambda_k = mu_k c_p,k/Pr, mixed by
 *             Eqs. muT_mix and conduct_mix with X_k = Y_k M/M_k.
 * Species diffusivity (constant-Lewis closure of j_k = -rho D_k grad Y_k):
 *             rho D_k = lambda/(c_p Le_k), c_p of the mixture.               */
static void mixture(const orc_setup* s, const double Phi[ORC_MAXS][ORC_MAXS], double T,
                    const double* Y, double* mu, double* lam, double* rhoD) {
    double mu0 = s->rho_in * s->nu_in * sutherland_ratio(s, T);
    if (s->transport == 0 || s->ns == 0) {
        *mu = mu0;
        *lam = mu0 * cp_of(s, Y) / s->Pr;
    } else {
        double X[ORC_MAXS], mbar = 1.0 / inv_mbar(s, Y);
        for (int k = 0; k < s->ns; ++k) X[k] = Y[k] * mbar / s->M[k];
        double m = 0.0, l1 = 0.0, l2 = 0.0;
        for (int k = 0; k < s->ns; ++k) {
            double muk = s->mu_star[k] * mu0;
            double lamk = muk * (s->cpk ? s->cp_k[k] : s->cp) / s->Pr;
            double den = 0.0;
            for (int j = 0; j < s->ns; ++j) den += Phi[k][j] * X[j];
            m += muk * X[k] / den;
            l1 += X[k] * lamk;
            l2 += X[k] / lamk;
        }
        *mu = m;
        *lam = 0.5 * (l1 + 1.0 / l2);
    }
    if (rhoD) {
        double cp = cp_of(s, Y);
        for (int k = 0; k < s->ns; ++k) rhoD[k] = *lam / (cp * s->Le[k]);
    }
}

static void build_phi(const orc_setup* s, double Phi[ORC_MAXS][ORC_MAXS]) {
    for (int k = 0; k < ORC_MAXS; ++k)
        for (int j = 0; j < ORC_MAXS; ++j) Phi[k][j] = 0.0;
    for (int k = 0; k < s->ns; ++k)
        for (int j = 0; j < s->ns; ++j)
            Phi[k][j] = wilke_phi(s->mu_star[k], s->mu_star[j], s->M[k], s->M[j]);
}

void orc_mixture(const orc_setup* s, double T, const double* Y, double* mu, double* lam,
                 double* rhoD) {
    double Phi[ORC_MAXS][ORC_MAXS];
    build_phi(s, Phi);
    mixture(s, Phi, T, Y, mu, lam, rhoD);
}

/* ------------------------------------------------------------- LB kernels */

void orc_lattice(int32_t dim, int32_t* c, double* w) {
    int Q = dim == 2 ? 9 : 19;
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = dim == 2 ? C2[i][a] : C3[i][a];
        w[i] = dim == 2 ? W2[i] : W3[i];
    }
}

/* Equilibrium and source of the pressure-based populations (Sec. 3.3,
 * Eqs. eq-pop-f, eq-pop-g, body-force):
 *   f_i^eq/rho = w_i (1 + e_i),  e_i = c.u/cs2 + (c.u)^2/(2 cs2^2) - u^2/(2 cs2)
 *   g_i^eq = cs2 f_i^eq + w_i (P_h - rho cs2)       = w_i (P_h + rho cs2 e_i)
 *   Xi_i = (c_i - u).[ grad(rho cs2)(f^eq/rho - w) + F f^eq/rho ] + rho cs2 w divu
 *        = (c_i - u).[ G w_i e_i + F w_i (1 + e_i) ] + rho cs2 w_i divu
 * with G = cs2 grad(rho) and F the total force on the fluid.  The right-hand
 * forms are the same expressions with rho w_i cancelled out.                 */
static void eq_source(int Q, const int (*c)[3], const double* w, double rho, const double* u,
                      double Ph, const double* G, const double* F, double divu, double* geq,
                      double* xi) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = c[i][0] * u[0] + c[i][1] * u[1] + c[i][2] * u[2];
        double e = cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
        geq[i] = w[i] * (Ph + rho * CS2 * e);
        if (xi) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                s += (c[i][a] - u[a]) * (G[a] * w[i] * e + F[a] * w[i] * (1.0 + e));
            xi[i] = s + rho * CS2 * w[i] * divu;
        }
    }
}

void orc_eq_source(int32_t dim, double rho, const double* u, double Ph, const double* G,
                   const double* F, double divu, double* geq, double* xi) {
    double uu[3] = {u[0], u[1], dim == 3 ? u[2] : 0.0};
    double GG[3] = {G[0], G[1], dim == 3 ? G[2] : 0.0};
    double FF[3] = {F[0], F[1], dim == 3 ? F[2] : 0.0};
    if (dim == 2)
        eq_source(9, C2, W2, rho, uu, Ph, GG, FF, divu, geq, xi);
    else
        eq_source(19, C3, W3, rho, uu, Ph, GG, FF, divu, geq, xi);
}

/* Macroscopic state of one cell from its post-stream populations.
 * Moment recovery for the discrete scheme gbar = g + (g - g^eq)/(2 tau) - Xi/2
 * (a standard second-order shift; the paper does not print it):
 *   m  = sum_i c_i gbar_i / cs2,  S0 = sum_i gbar_i
 *   rho u = m + F/2, with F = F_b + F_drag and the drag of Eq.
 *   Fdrag-empirical-law taken at the new velocity (u_solid = 0):
 *   F_drag = -K u,  K = A_u mu phi_f phi_s^2/eta^2  =>  u = (m + F_b/2)/(rho + K/2)
 *   P_h = S0 + (sum_i Xi_i)/2 = S0 + (u.G + rho cs2 divu)/2.                 */
static void lb_macro(const orc_ctx* o, const double* gb, double rho, double mu, double phis,
                     double divu, const double* G, double* u, double* F, double* Ph) {
    const orc_setup* s = &o->s;
    double S0 = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < o->Q; ++i) {
        S0 += gb[i];
        for (int a = 0; a < 3; ++a) m[a] += o->c[i][a] * gb[i];
    }
    double phif = 1.0 - phis;
    double K = s->A_u * mu * phif * phis * phis / (s->eta * s->eta);
    if (s->si) K = 0.0; /* SI mode: no interface drag */
    for (int a = 0; a < 3; ++a) {
        m[a] = m[a] / CS2;
        u[a] = (m[a] + 0.5 * s->F_b[a]) / (rho + 0.5 * K);
        F[a] = s->F_b[a] - K * u[a];
    }
    if (s->dim == 2) u[2] = F[2] = 0.0;
    *Ph = S0 + 0.5 * (u[0] * G[0] + u[1] * G[1] + u[2] * G[2] + rho * CS2 * divu);
}

/* ---------------------------------------------------- FD ghost-cell rules */
/* State (T, Y) at an in-domain cell or at a ghost one step outside a face.
 * Periodic faces wrap; Dirichlet ghosts carry the face value (cell-centred
 * ghost); zero-gradient ghosts copy the cell on the inside (the caller's
 * cell, which is the only in-domain neighbour of a ghost on one axis).
 * Sharp-interface mode: a solid cell seen from a fluid cell is a ghost that
 * holds the solid temperature T_s at its centre (a fixed-temperature wall
 * for conduction) and the fluid cell's own composition (no species flux
 * into the solid); every term that reads the neighbour (diffusion,
 * convection, the density gradient) sees that ghost.                         */
static void state_at(const orc_ctx* o, int x, int y, int z, int cx, int cy, int cz, double* T,
                     double* Y) {
    const orc_setup* s = &o->s;
    int p[3] = {x, y, z}, n[3] = {s->nx, s->ny, s->nz}, cc[3] = {cx, cy, cz};
    for (int a = 0; a < 3; ++a) {
        if (p[a] >= 0 && p[a] < n[a]) continue;
        int face = 2 * a + (p[a] < 0 ? 0 : 1);
        int kind = s->fd_bc[face];
        if (kind == ORC_FD_PERIODIC) {
            p[a] = (p[a] + n[a]) % n[a];
        } else if (kind == ORC_FD_DIRICHLET) {
            *T = s->fd_val[face][0];
            for (int k = 0; k < s->ns; ++k) Y[k] = s->fd_val[face][1 + k];
            return;
        } else {
            p[0] = cc[0];
            p[1] = cc[1];
            p[2] = cc[2];
            break;
        }
    }
    long id = cidx(o, p[0], p[1], p[2]);
    if (is_solid(o, id)) {
        long ic = cidx(o, cc[0], cc[1], cc[2]);
        *T = s->T_s;
        for (int k = 0; k < s->ns; ++k) Y[k] = o->Y[(long)k * o->N + ic];
        return;
    }
    *T = o->T[id];
    for (int k = 0; k < s->ns; ++k) Y[k] = o->Y[(long)k * o->N + id];
}

/* G = cs2 grad(rho) by second-order central differences; the neighbour
 * densities come from the EOS of the neighbour states (ghosts included).    */
static void grad_rho(const orc_ctx* o, int x, int y, int z, double* G) {
    const orc_setup* s = &o->s;
    double Tm, Tp, Ym[ORC_MAXS], Yp[ORC_MAXS];
    for (int a = 0; a < 3; ++a) {
        G[a] = 0.0;
        if (a >= s->dim) continue;
        int dx = a == 0, dy = a == 1, dz = a == 2;
        state_at(o, x - dx, y - dy, z - dz, x, y, z, &Tm, Ym);
        state_at(o, x + dx, y + dy, z + dz, x, y, z, &Tp, Yp);
        G[a] = CS2 * (orc_eos(s, Tp, Yp) - orc_eos(s, Tm, Ym)) / 2.0;
    }
}

/* ----------------------------------------------------------- LB phase */
/* Collision (Sec. 3.3, Eq. pop-g discretised with the shift above):
 *   gbar*_i = gbar_i - (gbar_i - g_i^eq)/tau + (1 - 1/(2 tau)) Xi_i,
 *   tau = mu/(rho cs2) + 1/2  (the paper's mu = rho cs2 (tau_r - 1/2)).     */
static void lb_collide_phase(orc_ctx* o) {
    const orc_setup* s = &o->s;
    long tau_bad = 0;
#pragma omp parallel for reduction(+ : tau_bad) schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = cidx(o, x, y, z);
                double gb[19], geq[19], xi[19], G[3], u[3], F[3], Ph, mu, lam;
                double Yc[ORC_MAXS];
                for (int k = 0; k < s->ns; ++k) Yc[k] = o->Y[(long)k * o->N + id];
                double rho = orc_eos(s, o->T[id], Yc);
                if (is_solid(o, id)) { /* SI mode: a solid cell holds no flow */
                    for (int i = 0; i < o->Q; ++i) o->gs[(long)i * o->N + id] = o->g[(long)i * o->N + id];
                    for (int a = 0; a < 3; ++a) o->u[(long)a * o->N + id] = 0.0;
                    o->Ph[id] = 0.0;
                    o->rho_n[id] = rho;
                    continue;
                }
                mixture(s, o->Phi, o->T[id], Yc, &mu, &lam, NULL);
                for (int i = 0; i < o->Q; ++i) gb[i] = o->g[(long)i * o->N + id];
                grad_rho(o, x, y, z, G);
                lb_macro(o, gb, rho, mu, o->phi[id], o->divu[id], G, u, F, &Ph);
                double tau = mu / (rho * CS2) + 0.5;
                if (!(tau > 0.5)) tau_bad++;
                eq_source(o->Q, o->c, o->w, rho, u, Ph, G, F, o->divu[id], geq, xi);
                for (int i = 0; i < o->Q; ++i)
                    o->gs[(long)i * o->N + id] =
                        gb[i] - (gb[i] - geq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * xi[i];
                for (int a = 0; a < 3; ++a) o->u[(long)a * o->N + id] = u[a];
                o->Ph[id] = Ph;
                o->rho_n[id] = rho;
            }
    o->diag[ORC_D_TAUBAD] += (double)tau_bad;
}

/* Pull streaming with the boundary rules.  A population whose upstream cell
 * x - c_i lies outside a non-periodic face is set from values the collision
 * computed at x itself (walls take precedence at corners):
 *   wall:            halfway bounce-back, gbar_i(x) = gbar*_opp(i)(x)
 *   velocity inlet:  g_i^eq(rho_in, u_in, P_h(x))
 *   pressure outlet: g_i^eq(rho(x), u(x), P_h = 0)
 *   characteristic outlet: g_i^eq(rho(x), u(x), P_out) with
 *                    P_out = w + rho(x) c_s u_x(x)
 * The paper uses no-slip walls, a prescribed inlet and an open
 * (non-reflecting) outlet.  The characteristic outlet follows the
 * one-dimensional characteristic analysis of Poinsot and Lele that the paper
 * cites: the amplitude of the wave entering through the outlet,
 * w = P - rho c_s u_x, is held (an outgoing wave, which carries
 * dP = rho c_s du_x, then leaves without reflection) and only relaxed
 * towards the far-field pressure P_h = 0,
 *   w^{n+1} = w^n - K P_h(x)^n,  K = sigma c_s (1 - Ma^2) / n_x,
 * with Ma = |u_in| / c_s and n_x the domain length; w starts at 0.          */
static void lb_stream_phase(orc_ctx* o) {
    const orc_setup* s = &o->s;
    int n[3] = {s->nx, s->ny, s->nz};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = cidx(o, x, y, z);
                if (is_solid(o, id)) { /* SI mode: nothing streams in a solid cell */
                    for (int i = 0; i < o->Q; ++i) o->g[(long)i * o->N + id] = o->gs[(long)i * o->N + id];
                    continue;
                }
                for (int i = 0; i < o->Q; ++i) {
                    int p[3] = {x - o->c[i][0], y - o->c[i][1], z - o->c[i][2]};
                    /* SI mode: a link to a solid cell is a halfway bounce-back wall */
                    int wall = solid_at(o, p[0], p[1], p[2]), inlet = 0, outlet = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] >= 0 && p[a] < n[a]) continue;
                        int face = 2 * a + (p[a] < 0 ? 0 : 1);
                        int kind = s->lb_bc[face];
                        if (kind == ORC_LB_PERIODIC)
                            p[a] = (p[a] + n[a]) % n[a];
                        else if (kind == ORC_LB_WALL)
                            wall = 1;
                        else if (kind == ORC_LB_INLET)
                            inlet = 1;
                        else
                            outlet = 1;
                    }
                    double val;
                    if (wall) {
                        val = o->gs[(long)o->opp[i] * o->N + id];
                    } else if (inlet || outlet) {
                        double ub[3], ph, rho, geq[19];
                        if (inlet) {
                            /* inlet velocity of this row (y, z): the profile if
                             * one is set, else the uniform u_in */
                            long r = (long)z * s->ny + y;
                            for (int a = 0; a < 3; ++a)
                                ub[a] = o->uprof ? o->uprof[(long)a * s->ny * s->nz + r] : s->u_in[a];
                            if (s->dim == 2) ub[2] = 0.0;
                            ph = o->Ph[id];
                            rho = s->rho_in;
                        } else {
                            for (int a = 0; a < 3; ++a) ub[a] = o->u[(long)a * o->N + id];
                            rho = o->rho_n[id];
                            ph = 0.0;
                            if (s->lb_bc[1] == ORC_LB_CHAR_OUTLET)
                                ph = o->wout[(long)z * s->ny + y] + rho * sqrt(CS2) * ub[0];
                        }
                        eq_source(o->Q, o->c, o->w, rho, ub, ph, NULL, NULL, 0.0, geq, NULL);
                        val = geq[i];
                    } else {
                        val = o->gs[(long)i * o->N + cidx(o, p[0], p[1], p[2])];
                    }
                    o->g[(long)i * o->N + id] = val;
                }
            }
    if (s->lb_bc[1] == ORC_LB_CHAR_OUTLET) {
        double uin2 = s->u_in[0] * s->u_in[0] + s->u_in[1] * s->u_in[1] + s->u_in[2] * s->u_in[2];
        double K = s->outlet_sigma * sqrt(CS2) * (1.0 - uin2 / CS2) / s->nx;
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y) {
                long id = cidx(o, s->nx - 1, y, z);
                if (!is_solid(o, id)) o->wout[(long)z * s->ny + y] -= K * o->Ph[id];
            }
    }
}

/* ----------------------------------------------------------- FD phase */
/* One explicit Euler step of the temperature and species equations
 * (Eqs. energy-transport-DI-version and volume-averaged-species-equation-5,
 * dt = dx = 1), with
 *   convection: first-order upwind,
 *     adv(q) = sum_a [ max(u_a,0)(q_c - q_{c-a}) + min(u_a,0)(q_{c+a} - q_c) ]
 *   diffusion: conservative central differences with arithmetic-mean face
 *     coefficients, flux(c,nb) = (k_c + k_nb)/2 (q_nb - q_c)
 *   interface heat exchange (Eq. diffusion-heat-flux-3) relaxing T toward the
 *     solid temperature: S_I = H (T_s - T), H = A_T lambda phi_f phi_s^2/eta^2
 *     (the printed sign, with alpha = fluid, would drive T away from T_s;
 *     the paper describes the term as holding the prescribed wall value).
 *   dP0/dt = 0 (open domain) and the c_p,k j_k term vanishes for the equal
 *     species heat capacities used here.
 *   species face flux when the Lewis numbers differ: a correction velocity
 *     keeps sum_k J_k = 0: J_k = (rhoD_k)_f dY_k - Y_k,f sum_m (rhoD_m)_f dY_m.
 * Also returns the thermal divergence q_T/T used by the next LB step (the
 * solver is compressible only through temperature changes).                 */
static void fd_cell(const orc_ctx* o, int x, int y, int z, const double* u, double* Tout,
                    double* Yout, double* qTout) {
    const orc_setup* s = &o->s;
    long id = cidx(o, x, y, z);
    int ns = s->ns;
    double Tc = o->T[id], Yc[ORC_MAXS], mu_c, lam_c, rD_c[ORC_MAXS];
    for (int k = 0; k < ns; ++k) Yc[k] = o->Y[(long)k * o->N + id];
    double rho_c = orc_eos(s, Tc, Yc);
    mixture(s, o->Phi, Tc, Yc, &mu_c, &lam_c, rD_c);
    double phis = o->phi[id], phif = 1.0 - phis;
    double H = s->A_T * lam_c * phif * phis * phis / (s->eta * s->eta);
    if (s->si) H = 0.0; /* SI mode: no interface heat exchange */

    double advT = 0.0, lapT = 0.0, advY[ORC_MAXS], J[ORC_MAXS], cpj = 0.0;
    for (int k = 0; k < ns; ++k) advY[k] = J[k] = 0.0;
    for (int a = 0; a < s->dim; ++a) {
        int dx = a == 0, dy = a == 1, dz = a == 2;
        double Tm, Tp, Ym[ORC_MAXS], Yp[ORC_MAXS];
        state_at(o, x - dx, y - dy, z - dz, x, y, z, &Tm, Ym);
        state_at(o, x + dx, y + dy, z + dz, x, y, z, &Tp, Yp);
        double up = u[a] > 0.0 ? u[a] : 0.0, un = u[a] < 0.0 ? u[a] : 0.0;
        advT += up * (Tc - Tm) + un * (Tp - Tc);
        if (s->cpk) {
            /* species heat flux (sum_k c_p,k j_k) . grad T with the cell's
             * diffusive fluxes j_k = -rho D_k dY_k (plus the correction
             * velocity's Y_k sum_m rho D_m dY_m for unequal Lewis numbers),
             * central differences over the two neighbours (ghosts included) */
            double gT = 0.5 * (Tp - Tm), gY[ORC_MAXS], sum = 0.0, f = 0.0;
            for (int k = 0; k < ns; ++k) {
                gY[k] = 0.5 * (Yp[k] - Ym[k]);
                sum += rD_c[k] * gY[k];
            }
            for (int k = 0; k < ns; ++k) {
                double jk = -rD_c[k] * gY[k];
                if (o->corr) jk += Yc[k] * sum;
                f += s->cp_k[k] * jk;
            }
            cpj += f * gT;
        }
        for (int k = 0; k < ns; ++k) advY[k] += up * (Yc[k] - Ym[k]) + un * (Yp[k] - Yc[k]);
        for (int side = 0; side < 2; ++side) {
            double Tn = side == 0 ? Tm : Tp;
            const double* Yn = side == 0 ? Ym : Yp;
            double mu_n, lam_n, rD_n[ORC_MAXS];
            mixture(s, o->Phi, Tn, Yn, &mu_n, &lam_n, rD_n);
            lapT += 0.5 * (lam_c + lam_n) * (Tn - Tc);
            double Df[ORC_MAXS], dY[ORC_MAXS], sum = 0.0;
            for (int k = 0; k < ns; ++k) {
                Df[k] = 0.5 * (rD_c[k] + rD_n[k]);
                dY[k] = Yn[k] - Yc[k];
                sum += Df[k] * dY[k];
            }
            for (int k = 0; k < ns; ++k) {
                double Jk = Df[k] * dY[k];
                if (o->corr) Jk -= 0.5 * (Yc[k] + Yn[k]) * sum;
                J[k] += Jk;
            }
        }
    }
    double cp_c = cp_of(s, Yc);
    double qT = (lapT + H * (s->T_s - Tc) - cpj) / (rho_c * cp_c);
    double dlnp = 0.0;
    if (s->closed) {
        /* dP0/dt (Eq. energy-transport-DI-version), explicit: the change of
         * P0 over the previous step, P0_in (p^n - p^{n-1}) per unit time */
        const double mbar_in = ns ? 1.0 / inv_mbar(s, s->Y_in) : 1.0;
        const double P0_in = s->rho_in * s->r_gas * s->T_in / mbar_in;
        qT += P0_in * (s->p0 - o->p_prev) / (rho_c * cp_c);
        dlnp = (s->p0 - o->p_prev) / s->p0;
    }
    *Tout = Tc + (qT - advT);
    for (int k = 0; k < ns; ++k) Yout[k] = Yc[k] + (J[k] / rho_c - advY[k]);
    /* thermal divergence (1/T) DT/Dt, less (1/P0) dP0/dt in a closed domain */
    *qTout = qT / Tc - dlnp;
}

static void fd_phase(orc_ctx* o, int zero_u) {
    const orc_setup* s = &o->s;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = cidx(o, x, y, z);
                double u[3] = {0.0, 0.0, 0.0}, Y[ORC_MAXS], T, q;
                if (is_solid(o, id)) { /* SI mode: the solid keeps its state */
                    o->Tst[id] = o->T[id];
                    for (int k = 0; k < s->ns; ++k)
                        o->Yst[(long)k * o->N + id] = o->Y[(long)k * o->N + id];
                    o->qT[id] = 0.0;
                    continue;
                }
                if (!zero_u)
                    for (int a = 0; a < s->dim; ++a) u[a] = o->u[(long)a * o->N + id];
                fd_cell(o, x, y, z, u, &T, Y, &q);
                o->Tst[id] = T;
                for (int k = 0; k < s->ns; ++k) o->Yst[(long)k * o->N + id] = Y[k];
                o->qT[id] = q;
            }
}

/* ----------------------------------------------------------- chemistry */
/* Production rates (Sec. 3.2.2, Eq. 8; Sec. 3.3, Eq. 9):
 *   omega_k = M_k sum_j s_kj Q_j,  s_kj = nu''_kj - nu'_kj
 *   omega_T = - sum_k dh_f,k omega_k
 * Rates of progress by the law of mass action with Arrhenius rate constants
 * (the paper takes them from its kinetics library; here they are plain
 * tables):  k_f = A T^beta exp(-theta/T),  k_r = k_f / exp(a + b/T),
 *   Q_j = k_f prod_k [X_k]^nu'_kj - k_r prod_k [X_k]^nu''_kj,  [X_k] = rho Y_k/M_k. */
static void rates(const orc_setup* s, double T, const double* Y, double rho, double* wk,
                  double* wT) {
    double X[ORC_MAXS];
    for (int k = 0; k < s->ns; ++k) {
        X[k] = rho * Y[k] / s->M[k];
        wk[k] = 0.0;
    }
    for (int j = 0; j < s->nr; ++j) {
        double kf = s->A[j] * pow(T, s->beta[j]) * exp(-s->theta[j] / T);
        double qf = kf, qr = 0.0;
        for (int k = 0; k < s->ns; ++k)
            for (int p = 0; p < s->nu_f[j][k]; ++p) qf *= X[k];
        if (s->rev[j]) {
            qr = kf / exp(s->lnKc_a[j] + s->lnKc_b[j] / T);
            for (int k = 0; k < s->ns; ++k)
                for (int p = 0; p < s->nu_r[j][k]; ++p) qr *= X[k];
        }
        double Qj = qf - qr;
        for (int k = 0; k < s->ns; ++k) wk[k] += (double)(s->nu_r[j][k] - s->nu_f[j][k]) * Qj;
    }
    double w = 0.0;
    for (int k = 0; k < s->ns; ++k) {
        wk[k] = s->M[k] * wk[k];
        w -= s->dhf[k] * wk[k];
    }
    *wT = w;
}

void orc_rates(const orc_setup* s, double T, const double* Y, double rho, double* wk,
               double* wT) {
    rates(s, T, Y, rho, wk, wT);
}

/* Right-hand side f of the reaction step and its Jacobian at fixed density:
 * with [X_m] = rho Y_m / M_m and the law of mass action,
 *   d Q_j / d[X_m] = k_f nu'_mj [X_m]^(nu'_mj - 1) prod_{l != m} [X_l]^nu'_lj
 *                  - k_r nu''_mj [X_m]^(nu''_mj - 1) prod_{l != m} [X_l]^nu''_lj
 *   d Q_j / dT     = Q_f,j dln k_f/dT - Q_r,j dln k_r/dT,
 *     dln k_f/dT = beta/T + theta/T^2,  dln k_r/dT = dln k_f/dT + b/T^2
 *     (k_r = k_f / exp(a + b/T)),
 * and f_k = (M_k/rho) sum_j s_kj Q_j, f_T = -sum_k dh_f,k f_k / cp:
 *   d f_k/d Y_m = (M_k/M_m) sum_j s_kj d Q_j/d[X_m],
 *   d f_k/dT    = (M_k/rho) sum_j s_kj d Q_j/dT,
 *   d f_T/d y   = -sum_k dh_f,k d f_k/d y / cp.                              */
static double ipow(double x, int n) {
    double r = 1.0;
    for (int p = 0; p < n; ++p) r *= x;
    return r;
}
void orc_rates_jacobian(const orc_setup* s, double T, const double* Y, double rho, double* f,
                        double* J) {
    int ns = s->ns, n = ns + 1;
    double X[ORC_MAXS], G[ORC_MAXS][ORC_MAXS], GT[ORC_MAXS], w[ORC_MAXS];
    for (int k = 0; k < ns; ++k) {
        X[k] = rho * Y[k] / s->M[k];
        w[k] = GT[k] = 0.0;
        for (int m = 0; m < ns; ++m) G[k][m] = 0.0;
    }
    for (int j = 0; j < s->nr; ++j) {
        double kf = s->A[j] * pow(T, s->beta[j]) * exp(-s->theta[j] / T);
        double dlf = s->beta[j] / T + s->theta[j] / (T * T);
        double kr = s->rev[j] ? kf / exp(s->lnKc_a[j] + s->lnKc_b[j] / T) : 0.0;
        double dlr = dlf + s->lnKc_b[j] / (T * T);
        double qf = kf, qr = kr, dQ[ORC_MAXS];
        for (int k = 0; k < ns; ++k) {
            qf *= ipow(X[k], s->nu_f[j][k]);
            qr *= ipow(X[k], s->nu_r[j][k]);
        }
        for (int m = 0; m < ns; ++m) {
            double df = 0.0, dr = 0.0;
            if (s->nu_f[j][m] > 0) {
                df = kf * s->nu_f[j][m] * ipow(X[m], s->nu_f[j][m] - 1);
                for (int l = 0; l < ns; ++l)
                    if (l != m) df *= ipow(X[l], s->nu_f[j][l]);
            }
            if (s->rev[j] && s->nu_r[j][m] > 0) {
                dr = kr * s->nu_r[j][m] * ipow(X[m], s->nu_r[j][m] - 1);
                for (int l = 0; l < ns; ++l)
                    if (l != m) dr *= ipow(X[l], s->nu_r[j][l]);
            }
            dQ[m] = df - dr;
        }
        double Qj = qf - qr, dQT = qf * dlf - qr * dlr;
        for (int k = 0; k < ns; ++k) {
            double skj = (double)(s->nu_r[j][k] - s->nu_f[j][k]);
            if (skj == 0.0) continue;
            w[k] += skj * Qj;
            GT[k] += skj * dQT;
            for (int m = 0; m < ns; ++m) G[k][m] += skj * dQ[m];
        }
    }
    double fT = 0.0, cp = cp_of(s, Y); /* c_p held at the state's, like rho */
    for (int i = 0; i < n * n; ++i) J[i] = 0.0;
    for (int k = 0; k < ns; ++k) {
        f[k] = s->M[k] * w[k] / rho;
        fT -= s->dhf[k] * f[k] / cp;
        for (int m = 0; m < ns; ++m) J[k * n + m] = s->M[k] / s->M[m] * G[k][m];
        J[k * n + ns] = s->M[k] / rho * GT[k];
    }
    f[ns] = fT;
    for (int m = 0; m < n; ++m) {
        double v = 0.0;
        for (int k = 0; k < ns; ++k) v -= s->dhf[k] * J[k * n + m];
        J[ns * n + m] = v / cp;
    }
}

/* Solve A x = b in place (b becomes x) by Gaussian elimination with partial
 * pivoting; A (n x n, row-major) is overwritten.  Returns -1 for a singular A. */
static int lu_solve(int n, double* A, double* b) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return -1;
        if (p != c) {
            for (int q = 0; q < n; ++q) {
                double t = A[c * n + q];
                A[c * n + q] = A[p * n + q];
                A[p * n + q] = t;
            }
            double t = b[c];
            b[c] = b[p];
            b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double l = A[r * n + c] / A[c * n + c];
            for (int q = c; q < n; ++q) A[r * n + q] -= l * A[c * n + q];
            b[r] -= l * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double v = b[c];
        for (int q = c + 1; q < n; ++q) v -= A[c * n + q] * b[q];
        b[c] = v / A[c * n + c];
    }
    return 0;
}

/* Reaction sub-step after transport (Lie splitting; the paper's solver takes
 * its integrator from the kinetics library) of dY_k/dt = omega_k/rho,
 * dT/dt = omega_T/(rho cp) at constant pressure, over one time step:
 *   scheme 0: n_sub explicit Euler sub-steps, rho re-evaluated from the EOS
 *             at each;
 *   scheme 1: n_sub linearly implicit Euler (one-stage Rosenbrock) sub-steps
 *             of length h = 1/n_sub, (I - h J) dy = h f, y += dy, with f and
 *             J at the sub-step's state and density;
 *   scheme 2: n = min(n_sub, max(1, ceil(2 kappa))) explicit Euler sub-steps
 *             of length 1/n, kappa = max_i |J_ii| at the cell's state (the
 *             explicit step then keeps h kappa <= 1/2).                     */
static void chem_integrate(const orc_setup* s, double* T, double* Y) {
    double wk[ORC_MAXS], wT;
    int nsub = s->n_sub, ns = s->ns, n = ns + 1;
    if (s->chem_scheme == 1) {
        double h = 1.0 / nsub, f[ORC_MAXS + 1], J[(ORC_MAXS + 1) * (ORC_MAXS + 1)];
        for (int it = 0; it < nsub; ++it) {
            double rho = orc_eos(s, *T, Y);
            orc_rates_jacobian(s, *T, Y, rho, f, J);
            for (int i = 0; i < n * n; ++i) J[i] = -h * J[i];
            for (int i = 0; i < n; ++i) {
                J[i * n + i] += 1.0;
                f[i] *= h;
            }
            if (lu_solve(n, J, f) != 0) {
                *T = NAN;
                return;
            }
            for (int k = 0; k < ns; ++k) Y[k] += f[k];
            *T += f[ns];
        }
        return;
    }
    if (s->chem_scheme == 2) {
        double f[ORC_MAXS + 1], J[(ORC_MAXS + 1) * (ORC_MAXS + 1)], kap = 0.0;
        orc_rates_jacobian(s, *T, Y, orc_eos(s, *T, Y), f, J);
        for (int i = 0; i < n; ++i)
            if (fabs(J[i * n + i]) > kap) kap = fabs(J[i * n + i]);
        double m = ceil(2.0 * kap);
        nsub = m < 1.0 ? 1 : m > (double)s->n_sub ? s->n_sub : (int)m;
    }
    double h = 1.0 / nsub;
    for (int it = 0; it < nsub; ++it) {
        double rho = orc_eos(s, *T, Y), cp = cp_of(s, Y);
        rates(s, *T, Y, rho, wk, &wT);
        for (int k = 0; k < s->ns; ++k) Y[k] = Y[k] + h * wk[k] / rho;
        *T = *T + h * wT / (rho * cp);
    }
}

void orc_reactor(const orc_setup* s, double* T, double* Y, int32_t nsteps) {
    for (int n = 0; n < nsteps; ++n) chem_integrate(s, T, Y);
}

/* Per-cell reaction after the FD step; returns whether the cell is
 * reaction-active (|omega_T| dt/(rho cp) > theta_ign).  The new thermal
 * divergence adds the chemical temperature change to the transport part.   */
static void chem_phase(orc_ctx* o, int do_chem) {
    const orc_setup* s = &o->s;
    long flagged = 0;
#pragma omp parallel for reduction(+ : flagged) schedule(static)
    for (long id = 0; id < o->N; ++id) {
        double T = o->Tst[id], Y[ORC_MAXS], T0 = T;
        for (int k = 0; k < s->ns; ++k) Y[k] = o->Yst[(long)k * o->N + id];
        if (do_chem && s->ns > 0 && s->nr > 0 && !is_solid(o, id)) {
            double wk[ORC_MAXS], wT, rho = orc_eos(s, T, Y);
            rates(s, T, Y, rho, wk, &wT);
            if (fabs(wT) / (rho * cp_of(s, Y)) > s->theta_ign) flagged++;
            chem_integrate(s, &T, Y);
        }
        o->divu[id] = o->qT[id] + (T - T0) / T0;
        o->T[id] = T;
        for (int k = 0; k < s->ns; ++k) o->Y[(long)k * o->N + id] = Y[k];
    }
    o->diag[ORC_D_FLAGGED] += (double)flagged;
}

/* ----------------------------------------------------------- reductions */
/* Conservation diagnostics of the state at the end of the step:
 *   mass = sum rho, species = sum rho Y_k, enthalpy = sum rho (cp T + sum_k dh_f,k Y_k)
 * kinetic energy and max |u| from the step's LB velocity (with its rho),
 * extrema of T, and cumulative counters.                                     */
static void reduce_phase(orc_ctx* o, int count) {
    const orc_setup* s = &o->s;
    double mass = 0.0, sp[ORC_MAXS] = {0}, ent = 0.0, kin = 0.0, umax = 0.0;
    double Tmin = INFINITY, Tmax = -INFINITY;
    long nonfin = 0, negy = 0;
    for (long id = 0; id < o->N; ++id) {
        double Y[ORC_MAXS], T = o->T[id];
        for (int k = 0; k < s->ns; ++k) Y[k] = o->Y[(long)k * o->N + id];
        double rho = orc_eos(s, T, Y);
        double hsum = cp_of(s, Y) * T;
        int bad = !isfinite(T), neg = 0;
        for (int k = 0; k < s->ns; ++k) {
            sp[k] += rho * Y[k];
            hsum += s->dhf[k] * Y[k];
            if (!isfinite(Y[k])) bad = 1;
            if (Y[k] < -1e-12) neg = 1;
        }
        mass += rho;
        ent += rho * hsum;
        double uu = 0.0;
        for (int a = 0; a < s->dim; ++a) {
            double ua = o->u[(long)a * o->N + id];
            uu += ua * ua;
            if (!isfinite(ua)) bad = 1;
        }
        kin += 0.5 * o->rho_n[id] * uu;
        if (sqrt(uu) > umax) umax = sqrt(uu);
        if (T < Tmin) Tmin = T;
        if (T > Tmax) Tmax = T;
        nonfin += bad;
        negy += neg;
    }
    o->diag[ORC_D_MASS] = mass;
    for (int k = 0; k < ORC_MAXS; ++k) o->diag[ORC_D_SPECIES + k] = k < s->ns ? sp[k] : 0.0;
    o->diag[ORC_D_ENTHALPY] = ent;
    o->diag[ORC_D_KINETIC] = kin;
    o->diag[ORC_D_UMAX] = umax;
    o->diag[ORC_D_TMIN] = Tmin;
    o->diag[ORC_D_TMAX] = Tmax;
    if (count) {
        o->diag[ORC_D_NONFINITE] += (double)nonfin;
        o->diag[ORC_D_NEGY] += (double)negy;
    }
}

/* ----------------------------------------------------------------- API */

orc_ctx* orc_create(const orc_setup* s, const double* phi_solid) {
    if (!s || (s->dim != 2 && s->dim != 3) || s->nx < 2 || s->ny < 1 || s->nz < 1) return NULL;
    if (s->dim == 2 && s->nz != 1) return NULL;
    if (s->ns < 0 || s->ns > ORC_MAXS || s->nr < 0 || s->nr > ORC_MAXR || s->n_sub < 1)
        return NULL;
    orc_ctx* o = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    o->s = *s;
    o->Q = s->dim == 2 ? 9 : 19;
    o->N = (long)s->nx * s->ny * s->nz;
    o->c = s->dim == 2 ? C2 : C3;
    o->w = s->dim == 2 ? W2 : W3;
    for (int i = 0; i < o->Q; ++i)
        for (int j = 0; j < o->Q; ++j)
            if (o->c[i][0] == -o->c[j][0] && o->c[i][1] == -o->c[j][1] &&
                o->c[i][2] == -o->c[j][2])
                o->opp[i] = j;
    o->Mbar_in = s->ns > 0 ? 1.0 / inv_mbar(s, s->Y_in) : 1.0;
    build_phi(s, o->Phi);
    o->corr = 0;
    for (int k = 1; k < s->ns; ++k)
        if (s->Le[k] != s->Le[0]) o->corr = 1;
    long N = o->N;
    int ns = s->ns > 0 ? s->ns : 1;
    o->phi = (double*)calloc(N, sizeof(double));
    o->g = (double*)calloc(o->Q * N, sizeof(double));
    o->gs = (double*)calloc(o->Q * N, sizeof(double));
    o->T = (double*)calloc(N, sizeof(double));
    o->Y = (double*)calloc(ns * N, sizeof(double));
    o->divu = (double*)calloc(N, sizeof(double));
    o->u = (double*)calloc(3 * N, sizeof(double));
    o->Ph = (double*)calloc(N, sizeof(double));
    o->rho_n = (double*)calloc(N, sizeof(double));
    o->Tst = (double*)calloc(N, sizeof(double));
    o->Yst = (double*)calloc(ns * N, sizeof(double));
    o->qT = (double*)calloc(N, sizeof(double));
    o->wout = (double*)calloc((size_t)s->ny * s->nz, sizeof(double));
    if (phi_solid) memcpy(o->phi, phi_solid, N * sizeof(double));
    return o;
}

void orc_destroy(orc_ctx* o) {
    if (!o) return;
    free(o->phi); free(o->g); free(o->gs); free(o->T); free(o->Y); free(o->divu);
    free(o->u); free(o->Ph); free(o->rho_n); free(o->Tst); free(o->Yst); free(o->qT);
    free(o->uprof);
    free(o->wout);
    free(o);
}

/* Initial state: rho from the EOS, divu = 0, P_h = 0 and populations at
 * equilibrium, gbar = g^eq(rho, u, P_h = 0) (the half-step source shift is
 * not applied at t = 0).                                                     */
int orc_init_state(orc_ctx* o, const double* T, const double* Y, const double* u) {
    const orc_setup* s = &o->s;
    o->s.p0 = 1.0; /* a closed domain starts at P0 = P0_in */
    memset(o->wout, 0, (size_t)s->ny * s->nz * sizeof(double));
    o->p_prev = 1.0;
    for (long id = 0; id < o->N; ++id) {
        double Yc[ORC_MAXS], uc[3] = {0.0, 0.0, 0.0}, geq[19];
        o->T[id] = T[id];
        for (int k = 0; k < s->ns; ++k) Yc[k] = o->Y[(long)k * o->N + id] = Y[(long)k * o->N + id];
        if (u)
            for (int a = 0; a < s->dim; ++a) uc[a] = u[(long)a * o->N + id];
        double rho = orc_eos(s, T[id], Yc);
        eq_source(o->Q, o->c, o->w, rho, uc, 0.0, NULL, NULL, 0.0, geq, NULL);
        for (int i = 0; i < o->Q; ++i) o->g[(long)i * o->N + id] = geq[i];
        o->divu[id] = 0.0;
        for (int a = 0; a < 3; ++a) o->u[(long)a * o->N + id] = uc[a];
        o->rho_n[id] = rho;
    }
    for (int k = 0; k < ORC_D_LEN; ++k) o->diag[k] = 0.0;
    reduce_phase(o, 0); /* snapshot sums of the initial state; counters start at zero */
    o->S0 = s->closed ? closed_sum(o) : 0.0;
    return 0;
}

int orc_set_inlet_profile(orc_ctx* o, const double* u) {
    const orc_setup* s = &o->s;
    long nr = (long)s->ny * s->nz;
    free(o->uprof);
    o->uprof = NULL;
    if (!u) return 0;
    o->uprof = (double*)calloc(3 * nr, sizeof(double));
    for (int a = 0; a < s->dim; ++a)
        for (long r = 0; r < nr; ++r) o->uprof[a * nr + r] = u[a * nr + r];
    return 0;
}

int orc_set_populations(orc_ctx* o, const double* g, const double* divu) {
    memcpy(o->g, g, (size_t)o->Q * o->N * sizeof(double));
    if (divu) memcpy(o->divu, divu, o->N * sizeof(double));
    return 0;
}

int orc_step(orc_ctx* o, int32_t n, int32_t mask) {
    for (int it = 0; it < n; ++it) {
        if (mask & ORC_PH_LB) {
            lb_collide_phase(o);
            lb_stream_phase(o);
        } else {
            for (long i = 0; i < 3 * o->N; ++i) o->u[i] = 0.0;
            for (long id = 0; id < o->N; ++id) {
                double Yc[ORC_MAXS];
                for (int k = 0; k < o->s.ns; ++k) Yc[k] = o->Y[(long)k * o->N + id];
                o->rho_n[id] = orc_eos(&o->s, o->T[id], Yc);
            }
        }
        if (mask & ORC_PH_FD) {
            fd_phase(o, 0);
        } else {
            memcpy(o->Tst, o->T, o->N * sizeof(double));
            if (o->s.ns) memcpy(o->Yst, o->Y, (size_t)o->s.ns * o->N * sizeof(double));
            memset(o->qT, 0, o->N * sizeof(double));
        }
        chem_phase(o, (mask & ORC_PH_CHEM) != 0);
        reduce_phase(o, 1);
        o->diag[ORC_D_STEP] += 1.0;
        if (o->s.closed) {  /* P0 of the new state, for the next step */
            o->p_prev = o->s.p0;
            o->s.p0 = o->S0 / closed_sum(o);
        }
    }
    return 0;
}

double orc_p0(const orc_ctx* o) { return o->s.closed ? o->s.p0 : 1.0; }

int orc_fd_only(orc_ctx* o, double* Tstar, double* Ystar) {
    fd_phase(o, 1);
    memcpy(Tstar, o->Tst, o->N * sizeof(double));
    if (o->s.ns) memcpy(Ystar, o->Yst, (size_t)o->s.ns * o->N * sizeof(double));
    return 0;
}

/* Reads.  rho is the EOS of the current state; u and P_h are the moments of
 * the current post-stream populations (what the next step's collision uses). */
int orc_read(const orc_ctx* o, int32_t field, int32_t comp, double* out) {
    const orc_setup* s = &o->s;
    switch (field) {
    case ORC_F_T:
        memcpy(out, o->T, o->N * sizeof(double));
        return 0;
    case ORC_F_Y:
        if (comp < 0 || comp >= s->ns) return -1;
        memcpy(out, o->Y + (long)comp * o->N, o->N * sizeof(double));
        return 0;
    case ORC_F_DIVU:
        memcpy(out, o->divu, o->N * sizeof(double));
        return 0;
    case ORC_F_OUTW:
        memcpy(out, o->wout, (size_t)s->ny * s->nz * sizeof(double));
        return 0;
    case ORC_F_POP:
        if (comp < 0 || comp >= o->Q) return -1;
        memcpy(out, o->g + (long)comp * o->N, o->N * sizeof(double));
        return 0;
    case ORC_F_RHO:
    case ORC_F_U:
    case ORC_F_PH:
        if (field == ORC_F_U && (comp < 0 || comp >= s->dim)) return -1;
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y)
                for (int x = 0; x < s->nx; ++x) {
                    long id = cidx(o, x, y, z);
                    double Yc[ORC_MAXS], gb[19], G[3], u[3], F[3], Ph, mu, lam;
                    for (int k = 0; k < s->ns; ++k) Yc[k] = o->Y[(long)k * o->N + id];
                    double rho = orc_eos(s, o->T[id], Yc);
                    if (field == ORC_F_RHO) {
                        out[id] = rho;
                        continue;
                    }
                    if (is_solid(o, id)) { /* SI mode: a solid cell is at rest */
                        out[id] = 0.0;
                        continue;
                    }
                    mixture(s, o->Phi, o->T[id], Yc, &mu, &lam, NULL);
                    for (int i = 0; i < o->Q; ++i) gb[i] = o->g[(long)i * o->N + id];
                    grad_rho(o, x, y, z, G);
                    lb_macro(o, gb, rho, mu, o->phi[id], o->divu[id], G, u, F, &Ph);
                    out[id] = field == ORC_F_U ? u[comp] : Ph;
                }
        return 0;
    }
    return -1;
}

void orc_diag(const orc_ctx* o, double* out) {
    memcpy(out, o->diag, ORC_D_LEN * sizeof(double));
}

int32_t orc_nthreads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
