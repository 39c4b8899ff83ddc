// lbfd_device.h -- device-side data and per-cell arithmetic of the fused
// coupled step for gfx950.  Included by the kernel translation units (one per
// precision) and, for the parameter block layout only, by the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfd {

// array extent for a compile-time species bound (zero-length arrays are not allowed)
#define LBFD_NA(n) ((n) > 0 ? (n) : 1)

constexpr int MAXS = 16;
constexpr int MAXR = 32;
constexpr int MAXR_TAB = MAXR + 2;  // reaction table entries: two segments, each padded to pairs
constexpr int BLOCK = 256;       // threads per workgroup: 4 wave64
constexpr int DIAG_STRIDE = 32;  // doubles of partials per workgroup
constexpr int FLAG_GROUP = 4 * BLOCK;  // FP64-island mask words per scan group
constexpr int GSPREAD = 16;            // counters per group (word w adds to counter w % GSPREAD)
constexpr int ISLAND_WG = 1024;        // workgroups (and diagnostics slots) of the island
constexpr int MLP_SLOT_WG = 1024;      // most surrogate workgroups (two diagnostics slots each)
enum {
    DG_MASS = 0, DG_SP = 1, DG_ENTH = 17, DG_KIN = 18, DG_UMAX = 19, DG_TMIN = 20,
    DG_TMAX = 21, DG_NONFIN = 22, DG_TAUBAD = 23, DG_NEGY = 24, DG_FLAG = 25, DG_FALLBACK = 26,
    DG_FB_REASON = 27,  // four counters: envelope, overdraw, residual, positivity
    DG_COUNT = 31
};
static_assert(DG_COUNT <= DIAG_STRIDE, "diagnostic slot layout");
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_INLET = 2, BC_OUTLET = 3, BC_CHAR_OUTLET = 4 };
enum { FD_PERIODIC = 0, FD_DIRICHLET = 1, FD_NEUMANN = 2 };
enum { PH_LB = 1, PH_FD = 2, PH_CHEM = 4 };

// The reactions, one array per field (so that the data of consecutive
// reactions are adjacent and load together): Arrhenius data (in the FP32
// table theta, lnKc_a and lnKc_b are scaled by log2(e), so that the kernels
// exponentiate in base 2 and beta multiplies log2 T; an irreversible
// reaction has lnKc_a = +inf, so its reverse term is exactly zero); the species of each side's concentration product as four 8-bit
// indices (ascending; a species of order 2 appears twice; unused slots hold
// the species bound, whose concentration slot is 1); the net stoichiometric
// coefficients nu'' - nu' as numbers.  Two segments: entries [0, n_lo) are
// the reactions whose sides have at most two factors (evaluated with two),
// then [n_lo, n_tab) the others (four), each in the mechanism's order and
// padded to the kernel's reaction group with inert entries (A = 0).
template <typename R>
struct Rxn {
    R A[MAXR_TAB], beta[MAXR_TAB], theta[MAXR_TAB], lnKc_a[MAXR_TAB], lnKc_b[MAXR_TAB];
    uint32_t fidx[MAXR_TAB], ridx[MAXR_TAB];
    int32_t rev[MAXR_TAB];
    R nud[MAXR_TAB][MAXS];
};

// Every constant the kernels read, in the kernel's arithmetic type.  Lives in
// the device workspace and is read with wave-uniform (scalar) loads.
template <typename R>
struct Par {
    int nx, ny, nz, ns, nr;
    int n_lo, n_tab;  // reaction table segments (see Rxn)
    int n_sub, mu_model, transport, corr, any_beta;
    int chem_scheme;  // 0 explicit, 1 linearly implicit Euler, 2 adaptive explicit
    int lb_bc[6], fd_bc[6];
    R A_u, A_T, inv_eta2, T_s, cp, inv_cp, inv_Pr, rho_in, T_in, mu_ref, S_T_in, S;
    R rho_ref;        // rho_in * T_in / Mbar_in  (EOS numerator), times P0 / P0_in
                      // in a closed domain (rewritten on the device after each step)
    R p0;             // closed domain: P0 / P0_in of the step (1 otherwise); scales
                      // the single-gas EOS (with species it is in rho_ref)
    R dp0_term;       // closed domain: P0_in (p^n - p^{n-1}), the dP0/dt of the step
    R dlnp0;          // closed domain: (p^n - p^{n-1}) / p^n
    R inv_T_in;       // 1 / T_in, rounded once on the host
    R T_ref;          // the temperature planes hold T - T_ref: T_solid in FP32 mode
                      // (cells inside the particles sit at T_solid, where the
                      // stored offset is then exact to far below a kelvin's ulp),
                      // 0 in FP64 mode (the planes hold T itself)
    R Ts_rel;         // T_solid - T_ref
    R theta_ign, h_sub;
    R u_in[3], F_b[3];
    R inlet_eq[19];   // rho_in c_s^2 e_j(u_in): the inlet equilibria less their P_h part
    int char_out;     // +x face is the characteristic (non-reflecting) outlet
    R K_out;          // its relaxation factor sigma c_s (1 - Ma^2) / nx
    R c_s;            // sqrt(1/3), rounded once on the host
    R fd_face[6][1 + MAXS];  // Dirichlet face values: T - T_ref, then Y_k
    R rD_fac[MAXS];   // 1/(cp Le_k); with species heat capacities 1/Le_k (rho D_k =
                      // lambda/(c_p Le_k) with the cell's mixture c_p)
    int cpk;          // species heat capacities given (c_p = sum_k Y_k c_p,k)
    R cp_k[MAXS];     // c_p,k (0 for padding species)
    R M[MAXS], invM[MAXS], dhf[MAXS], mu_star[MAXS];
    R inv_mu_star[MAXS];  // 1 / mu_star (mu_star = 1 for padding species)
    R Pr_over_cp;         // Pr / cp
    R Phi[MAXS][MAXS];
    Rxn<R> rx;
};

// ------------------------------------------------------------------ lattice
template <int D> struct Lat;
// In FP32 mode the populations are stored scaled by 36 (G_i = 36 g_i): the
// lattice weights then become the small integers k_i = 36 w_i, exact in FP32,
// so that the collision's sums over the directions reproduce the weights'
// moments exactly (sum w = 1, sum w c c = cs^2 I).  With the weights rounded
// to FP32 (their sum is 1 + 1.5e-8 in D3Q19) every FP32 collision added a
// small pressure and momentum bias of the same sign, and after 1000 steps the
// velocity had drifted by up to 2e-5 of its maximum.  FP64 mode stores g
// itself with the weights in FP64.
template <> struct Lat<2> {
    static constexpr int Q = 9;
    static constexpr int k[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};
template <> struct Lat<3> {
    static constexpr int Q = 19;
    static constexpr int k[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// Direction of the FD face f (2 axis + side, side 0 = minus): the axis
// directions come first in both lattices, +axis then -axis.
__host__ __device__ constexpr int face_dir(int f) { return (f ^ 1) + 1; }
static_assert(Lat<3>::cx[face_dir(0)] == -1 && Lat<3>::cx[face_dir(1)] == 1 &&
                  Lat<3>::cy[face_dir(2)] == -1 && Lat<3>::cy[face_dir(3)] == 1 &&
                  Lat<3>::cz[face_dir(4)] == -1 && Lat<3>::cz[face_dir(5)] == 1 &&
                  Lat<2>::cx[face_dir(0)] == -1 && Lat<2>::cy[face_dir(3)] == 1,
              "face directions");

// Sharp-interface mode: per-cell link mask.  Bit i (1 <= i < Q) is set when
// the cell x + c_i (after periodic wrapping; none beyond a non-periodic face)
// is solid, bit SI_SELF when the cell itself is.  A cell is solid when its
// phase field is at least 1/2 (decided on the host in FP64).
constexpr uint32_t SI_SELF = 1u << 31;

// Stored populations = scale * g: 36 in FP32 mode, 1 in FP64 mode.
template <typename R>
struct Pop {
    static constexpr double scale = sizeof(R) == 4 ? 36.0 : 1.0;
    static constexpr double inv = sizeof(R) == 4 ? 1.0 / 36.0 : 1.0;  // S0 = inv sum
    static constexpr double mom = sizeof(R) == 4 ? 3.0 / 36.0 : 3.0;  // m = mom sum c
};
// The weight of direction i on the stored scale: the integer 36 w_i in FP32
// mode, w_i in FP64 mode.
template <typename R, int D>
__host__ __device__ constexpr double pop_w(int i) {
    return sizeof(R) == 4 ? (double)Lat<D>::k[i] : Lat<D>::w[i];
}

// ------------------------------------------------------------- arithmetic
// FP32 mode uses the hardware reciprocal / square root / exp2 / log2
// (about 1 ulp); the FP64 mode uses correctly rounded division and the
// device library's exp and log.
template <typename R> __device__ __forceinline__ R rcp(R x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename R> __device__ __forceinline__ R dvd(R a, R b);
template <> __device__ __forceinline__ float dvd<float>(float a, float b) {
    return a * __builtin_amdgcn_rcpf(b);
}
template <> __device__ __forceinline__ double dvd<double>(double a, double b) { return a / b; }
template <typename R> __device__ __forceinline__ R fsqrt(R x);
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }
template <typename R> __device__ __forceinline__ R fexp(R x);
template <> __device__ __forceinline__ float fexp<float>(float x) { return __expf(x); }
template <> __device__ __forceinline__ double fexp<double>(double x) { return exp(x); }
template <typename R> __device__ __forceinline__ R flog(R x);
template <> __device__ __forceinline__ float flog<float>(float x) { return __logf(x); }
template <> __device__ __forceinline__ double flog<double>(double x) { return log(x); }

// ----------------------------------------------------------------- closures
// Ideal-gas density at fixed thermodynamic pressure: rho = rho_in (T_in/T)(M/M_in).
// The sums run over the kernel's species bucket: a padding species has Y = 0
// and 1/M = 0, so it adds an exact zero (no branch on the species count).
template <typename R, int NSM>
__device__ __forceinline__ R eos(const Par<R>& P, R T, const R* Y) {
    if constexpr (NSM == 0) {
        return P.p0 * (P.rho_in * dvd(P.T_in, T));
    } else {
        R im = R(0);
#pragma unroll
        for (int k = 0; k < NSM; ++k) im += Y[k] * P.invM[k];
        return dvd(P.rho_ref, T * im);
    }
}

// Sutherland law as a ratio to the inlet viscosity.
template <typename R>
__device__ __forceinline__ R sutherland(const Par<R>& P, R T) {
    if (P.mu_model == 0) return R(1);
    // FP32: the reciprocal of the constant comes from the host (no per-cell
    // reciprocal); FP64: the division as written
    R x;
    if constexpr (sizeof(R) == 4)
        x = T * P.inv_T_in;
    else
        x = dvd(T, P.T_in);
    return dvd(x * fsqrt(x) * P.S_T_in, T + P.S);
}

// Mixture heat capacity c_p = sum_k Y_k c_p,k (kernels built with species
// heat capacities only).
template <typename R, int NSM>
__device__ __forceinline__ R cp_mix(const Par<R>& P, const R* Y) {
    R c = R(0);
#pragma unroll
    for (int k = 0; k < NSM; ++k) c += Y[k] * P.cp_k[k];
    return c;
}

// Viscosity and conductivity of one state (single gas or Wilke mixture).
// CPK: species heat capacities, lambda = mu c_p/Pr with the mixture c_p
// (single gas only; the runtime refuses them with the Wilke closure).
template <typename R, int NSM, bool CPK = false>
__device__ __forceinline__ void transport(const Par<R>& P, R T, const R* Y, R& mu, R& lam) {
    R mu0 = P.mu_ref * sutherland(P, T);
    if constexpr (NSM > 0) {
        if (P.transport != 0) {
            R X[LBFD_NA(NSM)], im = R(0);
#pragma unroll
            for (int k = 0; k < NSM; ++k) im += Y[k] * P.invM[k];
            R mbar = rcp(im);
#pragma unroll
            for (int k = 0; k < NSM; ++k) X[k] = Y[k] * mbar * P.invM[k];
            R m = R(0), l1 = R(0), l2 = R(0);
            // FP32: 1/lambda_k = (1/mu*_k) (1/mu0) (Pr/cp), one reciprocal per
            // state instead of one per species
            R inv_l0 = R(0);
            if constexpr (sizeof(R) == 4) inv_l0 = rcp(mu0) * P.Pr_over_cp;
            // The sums run over the species bucket: a padding species has
            // X = 0, mu* = 1 and a row of ones in Phi (its denominator is then
            // sum X = 1), so every term it adds is an exact zero.
#pragma unroll
            for (int k = 0; k < NSM; ++k) {
                R den = R(0);
#pragma unroll
                for (int j = 0; j < NSM; ++j) den += P.Phi[k][j] * X[j];
                R muk = P.mu_star[k] * mu0;
                R lamk = muk * P.cp * P.inv_Pr;
                m += dvd(muk * X[k], den);
                l1 += X[k] * lamk;
                if constexpr (sizeof(R) == 4)
                    l2 += X[k] * (P.inv_mu_star[k] * inv_l0);
                else
                    l2 += dvd(X[k], lamk);
            }
            mu = m;
            lam = R(0.5) * (l1 + rcp(l2));
            return;
        }
    }
    mu = mu0;
    if constexpr (CPK && NSM > 0)
        lam = mu0 * cp_mix<R, NSM>(P, Y) * P.inv_Pr;
    else
        lam = mu0 * P.cp * P.inv_Pr;
}

// e_i = c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2) with cs2 = 1/3
template <typename R>
__device__ __forceinline__ R eq_e(R cu, R uu) {
    return R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
}

// ---------------------------------------------------------------- chemistry
template <int V>
struct Int {
    static constexpr int value = V;
};

// The parameter block as the kernels see it: a generic reference whose
// pointer comes from the constant address space, so that every uniform read
// of it compiles to a scalar load (the block does not change during a launch).
template <typename T>
__device__ __forceinline__ const T& const_block(const T* p) {
    return *(const T*)(const __attribute__((address_space(4))) T*)(uintptr_t)p;
}

// Mass-action Arrhenius production rates (omega_k = M_k sum_j s_kj Q_j,
// omega_T = -sum_k dh_k omega_k), evaluated in type C.  The concentration
// products index the concentrations with the reaction's (uniform) species
// indices, which indexes registers directly; each factor multiplies in
// ascending species order, as the definition's product is written.  With
// nine or more species the reactions go in pairs, without a branch on
// reversibility, so that two reactions' table loads and exponentials overlap.
template <typename C, int NSM>
__device__ __forceinline__ void rates(const Par<C>& P, C T, const C* Y, C rho, C* wk, C& wT) {
    C X[NSM + 1];
#pragma unroll
    for (int k = 0; k < NSM; ++k) {
        X[k] = rho * Y[k] * P.invM[k];
        wk[k] = C(0);
    }
    X[NSM] = C(1);
    const C invT = rcp(T);
    // FP32: base-2 exponentials of the base-2 table; FP64: natural ones
    constexpr bool B2 = sizeof(C) == 4;
    C lgT = C(0);
    if (P.any_beta) {
        if constexpr (B2)
            lgT = __builtin_amdgcn_logf(T);
        else
            lgT = flog(T);
    }
    auto ex = [](C v) {
        if constexpr (B2)
            return __builtin_amdgcn_exp2f(v);
        else
            return fexp(v);
    };
    constexpr int G = NSM >= 9 ? 2 : 1;
    const Rxn<C>& r = P.rx;
    auto react = [&](int j, auto nfac) {
        constexpr int NF = decltype(nfac)::value;
        const C kf = r.A[j] * ex(r.beta[j] * lgT - r.theta[j] * invT);
        const uint32_t f = r.fidx[j];
        C Qj = kf;
#pragma unroll
        for (int q = 0; q < NF; ++q) Qj = Qj * X[(f >> (8 * q)) & 255u];
        if (G > 1 || r.rev[j]) {
            const uint32_t b = r.ridx[j];
            C qr = kf * ex(-(r.lnKc_a[j] + r.lnKc_b[j] * invT));
#pragma unroll
            for (int q = 0; q < NF; ++q) qr = qr * X[(b >> (8 * q)) & 255u];
            Qj -= qr;
        }
#pragma unroll
        for (int k = 0; k < NSM; ++k) wk[k] += r.nud[j][k] * Qj;
    };
    const int n_lo = P.n_lo, n_tab = P.n_tab;
    for (int j = 0; j < n_lo; j += G) {
#pragma unroll
        for (int u = 0; u < G; ++u) react(j + u, Int<2>{});
    }
    for (int j = n_lo; j < n_tab; j += G) {
#pragma unroll
        for (int u = 0; u < G; ++u) react(j + u, Int<4>{});
    }
    C w = C(0);
#pragma unroll
    for (int k = 0; k < NSM; ++k) {
        wk[k] = P.M[k] * wk[k];
        w -= P.dhf[k] * wk[k];
    }
    wT = w;
}

// 1 / c_p of a state: the mixture's with species heat capacities (CPK), the
// parameter otherwise.
template <typename C, int NSM, bool CPK>
__device__ __forceinline__ C inv_cp_of(const Par<C>& P, const C* Y) {
    if constexpr (CPK && NSM > 0)
        return C(1) / cp_mix<C, NSM>(P, Y);
    else
        return P.inv_cp;
}

// One explicit Euler sub-step from rates already evaluated at (T, Y, rho).
template <typename C, int NSM, bool CPK = false>
__device__ __forceinline__ void chem_apply(const Par<C>& P, C& T, C* Y, C rho, const C* wk, C wT) {
    const C hr = P.h_sub * rcp(rho);
    const C icp = inv_cp_of<C, NSM, CPK>(P, Y);
#pragma unroll
    for (int k = 0; k < NSM; ++k) Y[k] = Y[k] + hr * wk[k];
    T = T + hr * wT * icp;
}

// n_sub explicit Euler sub-steps at constant pressure, in type C.
template <typename C, int NSM, bool CPK = false>
__device__ __forceinline__ void chem_integrate(const Par<C>& P, C& T, C* Y) {
    C wk[LBFD_NA(NSM)], wT;
    for (int n = 0; n < P.n_sub; ++n) {
        const C rho = eos<C, NSM>(P, T, Y);
        rates<C, NSM>(P, T, Y, rho, wk, wT);
        chem_apply<C, NSM, CPK>(P, T, Y, rho, wk, wT);
    }
}

// The same n_sub sub-steps, carried as increments (dT, dY) on a fixed base
// state (T0, Y0): the sub-step state is T0 + dT, and the caller gets the
// increments at full precision (in FP32 the chemical heat release of a slow
// cell is far below the rounding unit of T).  `wk`, `wT` and `rho0` hold the
// rates already evaluated at the base state.
template <typename C, int NSM, bool CPK = false>
__device__ __forceinline__ void chem_increments(const Par<C>& P, C T0, const C* Y0, C rho0,
                                                const C* wk0, C wT0, C& dT, C* dY) {
    C hr = P.h_sub * rcp(rho0);
#pragma unroll
    for (int k = 0; k < NSM; ++k) dY[k] = hr * wk0[k];
    dT = hr * wT0 * inv_cp_of<C, NSM, CPK>(P, Y0);
    C wk[LBFD_NA(NSM)], wT, Y[LBFD_NA(NSM)];
    for (int n = 1; n < P.n_sub; ++n) {
        const C T = T0 + dT;
#pragma unroll
        for (int k = 0; k < NSM; ++k) Y[k] = Y0[k] + dY[k];
        const C rho = eos<C, NSM>(P, T, Y);
        rates<C, NSM>(P, T, Y, rho, wk, wT);
        hr = P.h_sub * rcp(rho);
        const C icp = inv_cp_of<C, NSM, CPK>(P, Y);
#pragma unroll
        for (int k = 0; k < NSM; ++k) dY[k] = dY[k] + hr * wk[k];
        dT = dT + hr * wT * icp;
    }
}

// ---------------------------------------------- stiff reaction schemes
// (FP64; species buckets up to 9.)  The right-hand side of the reaction step
// at fixed density, f = (omega_k/rho, omega_T/(rho cp)), and its analytic
// Jacobian J[i][m] = d f_i / d y_m, y = (Y_1 .. Y_NSM, T): by the law of mass
// action, d Q_j / d[X_m] is the rate constant times the product of the other
// factors of the side (each factor of the side in turn), d ln k_f / dT =
// (beta + theta/T)/T and d ln k_r / dT = d ln k_f / dT + b/T^2; then
// d f_k/d Y_m = (M_k/M_m) sum_j s_kj d Q_j/d[X_m], d f_k/dT = (M_k/rho)
// sum_j s_kj d Q_j/dT and row T = -sum_k dh_f,k (row k) / cp.
// One reaction's terms for the Jacobian: the net rate Q_j, its temperature
// derivative dQ_j/dT, and d Q_j / d[X_m] as the sum over the side factors q
// with species index fi[q] (forward) and ri[q] (reverse): each factor of a
// side contributes the product of the others (df[q], dr[q]); padding
// factors carry the index NSM (concentration 1).
template <int NSM>
struct RxnTerms {
    double Qj, dQT, df[4], dr[4];
    int fi[4], ri[4];
    // d Q_j / d[X_m]
    __device__ __forceinline__ double dQ(int m) const {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v += fi[q] == m ? df[q] : 0.0;
            v -= ri[q] == m ? dr[q] : 0.0;
        }
        return v;
    }
};
template <int NSM>
__device__ __forceinline__ RxnTerms<NSM> rxn_terms(const Par<double>& P, int j, const double* X,
                                                   double lgT, double invT) {
    const Rxn<double>& r = P.rx;
    RxnTerms<NSM> t;
    const int nf = j < P.n_lo ? 2 : 4;
    const double kf = r.A[j] * fexp(r.beta[j] * lgT - r.theta[j] * invT);
    const double dlf = (r.beta[j] + r.theta[j] * invT) * invT;
    const bool rv = r.rev[j] != 0;
    const double kr = rv ? kf * fexp(-(r.lnKc_a[j] + r.lnKc_b[j] * invT)) : 0.0;
    const double dlr = dlf + r.lnKc_b[j] * invT * invT;
    double xf[4], xr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        t.fi[q] = q < nf ? (int)((r.fidx[j] >> (8 * q)) & 255u) : NSM;
        t.ri[q] = q < nf ? (int)((r.ridx[j] >> (8 * q)) & 255u) : NSM;
        xf[q] = X[t.fi[q]];
        xr[q] = X[t.ri[q]];
    }
    const double qf = kf * xf[0] * xf[1] * xf[2] * xf[3];
    const double qr = kr * xr[0] * xr[1] * xr[2] * xr[3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double a = kf, b = kr;
#pragma unroll
        for (int o = 0; o < 4; ++o)
            if (o != q) {
                a *= xf[o];
                b *= xr[o];
            }
        t.df[q] = a;
        t.dr[q] = b;
    }
    t.Qj = qf - qr;
    t.dQT = qf * dlf - qr * dlr;
    return t;
}

template <int NSM>
__device__ __forceinline__ void rates_jacobian(const Par<double>& P, double T, const double* Y,
                                               double rho, double* f,
                                               double (&J)[NSM + 1][NSM + 1]) {
    constexpr int N1 = NSM + 1;
    // the sums over the reactions accumulate in the outputs and are scaled
    // in place afterwards: f[k] takes sum_j s_kj Q_j, J[k][m] sum_j s_kj
    // dQ_j/d[X_m] and J[k][NSM] sum_j s_kj dQ_j/dT
    double X[NSM + 1];
#pragma unroll
    for (int k = 0; k < NSM; ++k) {
        X[k] = rho * Y[k] * P.invM[k];
        f[k] = 0.0;
#pragma unroll
        for (int m = 0; m < N1; ++m) J[k][m] = 0.0;
    }
    X[NSM] = 1.0;
    const double invT = 1.0 / T;
    const double lgT = P.any_beta ? flog(T) : 0.0;
    for (int j = 0; j < P.n_tab; ++j) {
        const RxnTerms<NSM> t = rxn_terms<NSM>(P, j, X, lgT, invT);
        double dQ[NSM];
#pragma unroll
        for (int m = 0; m < NSM; ++m) dQ[m] = t.dQ(m);
#pragma unroll
        for (int k = 0; k < NSM; ++k) {
            const double s = P.rx.nud[j][k];
            f[k] += s * t.Qj;
            J[k][NSM] += s * t.dQT;
#pragma unroll
            for (int m = 0; m < NSM; ++m) J[k][m] += s * dQ[m];
        }
    }
    const double irho = 1.0 / rho;
    double fT = 0.0;
#pragma unroll
    for (int k = 0; k < NSM; ++k) {
        f[k] = P.M[k] * f[k] * irho;
        fT -= P.dhf[k] * f[k] * P.inv_cp;
#pragma unroll
        for (int m = 0; m < NSM; ++m) J[k][m] = P.M[k] * P.invM[m] * J[k][m];
        J[k][NSM] = P.M[k] * irho * J[k][NSM];
    }
    f[NSM] = fT;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NSM; ++k) v -= P.dhf[k] * J[k][m];
        J[NSM][m] = v * P.inv_cp;
    }
}

// The diagonal of the same Jacobian, d[i] = J[i][i], by the same arithmetic
// element for element (the adaptive scheme needs only its largest
// magnitude, and the full matrix would hold about 200 registers).
template <int NSM>
__device__ __forceinline__ void rates_jacobian_diag(const Par<double>& P, double T,
                                                    const double* Y, double rho, double* d) {
    double X[NSM + 1], G[NSM], GT[NSM];
#pragma unroll
    for (int k = 0; k < NSM; ++k) {
        X[k] = rho * Y[k] * P.invM[k];
        G[k] = GT[k] = 0.0;
    }
    X[NSM] = 1.0;
    const double invT = 1.0 / T;
    const double lgT = P.any_beta ? flog(T) : 0.0;
    for (int j = 0; j < P.n_tab; ++j) {
        const RxnTerms<NSM> t = rxn_terms<NSM>(P, j, X, lgT, invT);
#pragma unroll
        for (int k = 0; k < NSM; ++k) {
            const double s = P.rx.nud[j][k];
            GT[k] += s * t.dQT;
            G[k] += s * t.dQ(k);
        }
    }
    const double irho = 1.0 / rho;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < NSM; ++k) {
        d[k] = P.M[k] * P.invM[k] * G[k];
        v -= P.dhf[k] * (P.M[k] * irho * GT[k]);
    }
    d[NSM] = v * P.inv_cp;
}

// A x = b by Gaussian elimination with partial pivoting, b overwritten with
// x.  Every index is a compile-time constant after unrolling: the pivot row
// is swapped in with selects.
template <int n>
__device__ __forceinline__ void solve_pivoted(double (&A)[n][n], double (&b)[n]) {
#pragma unroll
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < n; ++r) {
            const double v = fabs(A[r][c]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
#pragma unroll
        for (int r = c + 1; r < n; ++r) {
            const bool sw = r == p;
#pragma unroll
            for (int q = c; q < n; ++q) {
                const double t = A[c][q];
                A[c][q] = sw ? A[r][q] : t;
                A[r][q] = sw ? t : A[r][q];
            }
            const double t = b[c];
            b[c] = sw ? b[r] : t;
            b[r] = sw ? t : b[r];
        }
#pragma unroll
        for (int r = c + 1; r < n; ++r) {
            const double l = A[r][c] / A[c][c];
#pragma unroll
            for (int q = c; q < n; ++q) A[r][q] -= l * A[c][q];
            b[r] -= l * b[c];
        }
    }
#pragma unroll
    for (int c = n - 1; c >= 0; --c) {
        double v = b[c];
#pragma unroll
        for (int q = c + 1; q < n; ++q) v -= A[c][q] * b[q];
        b[c] = v / A[c][c];
    }
}

// The reaction step of one time step in FP64, by the parameters' scheme:
//   0: n_sub explicit Euler sub-steps;
//   1: n_sub linearly implicit (one-stage Rosenbrock) Euler sub-steps,
//      (I - h J) dy = h f at the sub-step's state and density, y += dy;
//   2: n = min(n_sub, max(1, ceil(2 kappa))) explicit sub-steps of length
//      1/n, kappa = max_i |J_ii| at the cell's state.
// CS: the scheme fixed at compile time (1 or 2: a kernel carries only that
// scheme's registers), or -1 to take it from the parameters.
template <int NSM, int CS = -1>
__device__ __forceinline__ void chem_step(const Par<double>& P, double& T, double* Y) {
    if constexpr (NSM > 0 && NSM <= 9) {
        constexpr int N1 = NSM + 1;
        const int cs = CS >= 0 ? CS : P.chem_scheme;
        if (cs == 1) {
            // The temperature rows of J and f are -sum_k dh_k (species row
            // k) / c_p, so the system's temperature equation reduces exactly
            // to dT = sum_k c_k dY_k with c_k = -dh_k / c_p; substituted, it
            // leaves the species system (I - h (J_YY + J_YT c^T)) dY = h f_Y,
            // solved here in place of the full one (equal up to rounding).
            const double h = P.h_sub;
            for (int it = 0; it < P.n_sub; ++it) {
                double J[N1][N1], b[N1];
                rates_jacobian<NSM>(P, T, Y, eos<double, NSM>(P, T, Y), b, J);
                double A[NSM][NSM], r[NSM];
#pragma unroll
                for (int k = 0; k < NSM; ++k) {
#pragma unroll
                    for (int m = 0; m < NSM; ++m)
                        A[k][m] = -h * (J[k][m] - J[k][NSM] * (P.dhf[m] * P.inv_cp));
                    A[k][k] += 1.0;
                    r[k] = h * b[k];
                }
                solve_pivoted<NSM>(A, r);
                double dT = 0.0;
#pragma unroll
                for (int k = 0; k < NSM; ++k) {
                    Y[k] += r[k];
                    dT -= P.dhf[k] * P.inv_cp * r[k];
                }
                T += dT;
            }
            return;
        }
        if (cs == 2) {
            double d[N1], kap = 0.0;
            rates_jacobian_diag<NSM>(P, T, Y, eos<double, NSM>(P, T, Y), d);
#pragma unroll
            for (int i = 0; i < N1; ++i) kap = fmax(kap, fabs(d[i]));
            const double m = ceil(2.0 * kap);
            const int nsub = m < 1.0 ? 1 : m > (double)P.n_sub ? P.n_sub : (int)m;
            const double h = 1.0 / nsub;
            double wk[NSM], wT;
            for (int it = 0; it < nsub; ++it) {
                const double rho = eos<double, NSM>(P, T, Y);
                rates<double, NSM>(P, T, Y, rho, wk, wT);
#pragma unroll
                for (int k = 0; k < NSM; ++k) Y[k] = Y[k] + h * wk[k] / rho;
                T = T + h * wT / (rho * P.cp);
            }
            return;
        }
    }
    chem_integrate<double, NSM>(P, T, Y);
}

// ------------------------------------------------------------ kernel args
// Closed domain: P0 / P0_in = p = S0 / S with S = sum over cells of M / T (the
// domain's mass is fixed and rho is proportional to P0 M / T).
struct P0State {
    double S0, p, p_prev;  // sum M / T of the initial state; p of this and the last step
    double rho_ref0;       // rho_ref at p = 1
    double P0_in;          // rho_ref0 * r_gas
};
constexpr int P0_PARTS = 4096;  // workgroups (and partial sums) of the P0 sum

template <typename R>
struct StepArgs {
    R* g;                 // [Q][N] populations (AA layout)
    const R* T_cur;       // [N]
    R* T_nxt;             // [N]
    const R* Y_cur;       // [ns][N]
    R* Y_nxt;             // [ns][N]
    R* divu;              // [N] (read, then overwritten in place)
    const R* phi;         // [N] solid fraction
    const uint32_t* smask;     // [N] sharp-interface link masks (SI kernels only)
    const double* inlet_prof;  // [ny*nz][19] rho_in c_s^2 e_j(u_in(y, z)) per inlet row,
                               // or null: the uniform inlet_eq of the parameters
    double* outlet_w;          // [ny*nz] characteristic outlet: incoming wave amplitude
                               // per outlet row (read and rewritten by the row's cell)
    double* partials;     // [nblocks][DIAG_STRIDE]
    unsigned long long* flags;  // [nblocks][zc][waves] reaction-active cells (FP32 mode)
    const Par<R>* P;
    const Par<double>* PD;
    int N;
    int nblocks;          // real workgroups (grid may be padded to a multiple of 8)
    int nbx, nby;         // cell tiles along x and y
    int zc;               // planes per workgroup (z-march length)
    int odd;              // AA parity of this step
    int phase;            // PH_* mask
    int diag;             // write diagnostics partials
    double* mtpart;       // closed domain: [diagnostics slots] sum of M / T of the new
                          // state over each slot's cells (null in an open domain)
    int sur;              // FP32 surrogate mode: reactions left to the surrogate kernels
    int stiff;            // stiff reaction scheme (chem_scheme 1 or 2, 0 none): the FP64 step
                          // and island kernels built with it
    int cpk;              // species heat capacities: the kernels built with them
    int ext;              // extended boundaries (sharp-interface masks, inlet profile,
                          // characteristic outlet, Dirichlet faces on periodic axes)
    // FP32 mode: compaction of the cells flagged for the FP64 reaction step
    int* gtot;            // [groups][GSPREAD] flagged cells per group of mask words (added
                          // by the kernels that write the masks, cleared by the island)
    int* list;            // [N] flagged cell indices in mask order
    int* count;           // [1] number of listed cells
    int P_nx, P_ny;       // grid extents (for the list kernel)
    // base of every plane, filled per launch: separate kernel arguments keep
    // each plane's base in scalar registers, so an access costs one shared
    // 32-bit lane offset instead of a 64-bit vector address per plane
    R* gpl[19];               // populations, plane i
    const R* Ycp[MAXS];       // Y_cur, species k
    R* Ynp[MAXS];             // Y_nxt, species k
};

// Halo planes of one x face (the strided copies a slab decomposition along x
// exchanges): entry p of the list is field plane `plane[p]` at x = xs[p],
// cells (xs[p], y, z) <-> buf[p][z][y].
constexpr int HALO_MAX_PLANES = 24;
static_assert(HALO_MAX_PLANES >= 5 + 1 + MAXS, "halo plane table");
template <typename R>
struct HaloArgs {
    R* plane[HALO_MAX_PLANES];
    int xs[HALO_MAX_PLANES];
    int nplanes, nx, ny, nz;
    R* buf;
    int pack;  // 1: planes -> buf, 0: buf -> planes
};

template <typename R>
struct MacroArgs {
    const R* g;
    const R* T;
    const R* Y;
    const R* divu;
    const R* phi;
    const uint32_t* smask;  // sharp-interface link masks, or null
    double* out;          // [5][N]: rho, u_x, u_y, u_z, P_h
    const Par<R>* P;
    const Par<double>* PD;
    int N, nblocks, odd;
};

template <typename R>
struct InitArgs {
    R* g;
    const R* T;
    const R* Y;
    const double* u;      // [dim][N] or null
    R* divu;
    const Par<R>* P;
    int N;
};

}  // namespace lbfd
