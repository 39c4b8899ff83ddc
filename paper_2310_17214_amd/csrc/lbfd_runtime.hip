// lbfd_runtime.hip -- host runtime behind the C ABI of include/lbfd.h:
// validation, workspace carving, parameter tables, step sequencing on the
// caller's stream, field reads and the deterministic diagnostics reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "lbfd.h"
#include "lbfd_device.h"
#include "lbfd_launch.h"
#include "lbfd_mlp.h"

using namespace lbfd;

namespace {

struct HostMech {
    int ns = 0, nr = 0;
    std::vector<double> M, dhf, mu_star, A, beta, theta, lnKc_a, lnKc_b;
    std::vector<int> nu_f, nu_r, rev;
    std::vector<double> cp;  // species heat capacities (empty: all at params.cp)
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t g, T0, T1, Y0, Y1, divu, phi, part, mtpart, flags, gtot, list, count, p0, p0part, parf,
        pard, scratch, red, sw, sp, solid, smask, inlet, outw, total;
    int nslots;                   // diagnostics slots: step tiles, island workgroups, then
                                  // two per surrogate workgroup
    int ngroups;                  // groups of FP64-island mask words
    int nbx, nby, zc, nblocks, grid;  // step kernel: 64 x TH tiles of one plane,
                                      // grid padded to a multiple of the 8 XCDs
    int nlin;                     // one-cell-per-thread kernels
};

int lattice_q(int dim) { return dim == 2 ? 9 : 19; }
int nsm_bucket(int ns) { return ns == 0 ? 0 : ns <= 4 ? 4 : ns <= 9 ? 9 : 16; }

Layout make_layout(const lbfd_grid& gr) {
    Layout L;
    const size_t N = (size_t)gr.nx * gr.ny * gr.nz;
    const size_t s = gr.precision == LBFD_FP32 ? 4 : 8;
    const int Q = lattice_q(gr.dim);
    const int nsm = nsm_bucket(gr.n_species);
    const int th = gr.precision == LBFD_FP32 ? step_tile_h_f32(gr.dim, nsm)
                                             : step_tile_h_f64(gr.dim, nsm);
    const int tw = BLOCK / th;
    L.nbx = (gr.nx + tw - 1) / tw;
    L.nby = (gr.ny + th - 1) / th;
    L.zc = 1;
    L.nblocks = L.nbx * L.nby * gr.nz;
    L.grid = (L.nblocks + 7) / 8 * 8;
    L.nlin = (int)((N + BLOCK - 1) / BLOCK);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.g = take(Q * N * s);
    L.T0 = take(N * s);
    L.T1 = take(N * s);
    // species planes for the kernel's species bucket (planes past n_species stay zero)
    L.Y0 = take((size_t)nsm_bucket(gr.n_species) * N * s);
    L.Y1 = take((size_t)nsm_bucket(gr.n_species) * N * s);
    L.divu = take(N * s);
    L.phi = take(N * s);
    // the surrogate's slots exist where it can run (FP32 with species)
    const bool sur = gr.precision == LBFD_FP32 && gr.n_species > 0;
    L.nslots = L.nblocks + ISLAND_WG + (sur ? 2 * MLP_SLOT_WG : 0);
    L.part = take((size_t)L.nslots * DIAG_STRIDE * sizeof(double));
    L.mtpart = take((size_t)L.nslots * sizeof(double));
    const size_t nwords = (size_t)L.nblocks * (BLOCK / 64);
    L.flags = take(nwords * sizeof(unsigned long long));
    L.ngroups = (int)((nwords + FLAG_GROUP - 1) / FLAG_GROUP);
    L.gtot = take((size_t)L.ngroups * GSPREAD * sizeof(int));
    L.list = take(N * sizeof(int));
    L.count = take(sizeof(int));
    L.p0 = take(sizeof(P0State));
    L.p0part = take(2 * P0_PARTS * sizeof(double));
    L.parf = take(sizeof(Par<float>));
    L.pard = take(sizeof(Par<double>));
    L.scratch = take(5 * N * sizeof(double));
    L.red = take(64 * sizeof(double));
    L.sw = take(sizeof(SurWeights));  // chemistry surrogate: packed weights
    L.sp = take(sizeof(SurPar));
    // sharp-interface mode: per-cell solid flags and link masks; the inlet
    // profile's equilibria per inlet row
    L.solid = take(N);
    L.smask = take(N * sizeof(uint32_t));
    L.inlet = take((size_t)gr.ny * gr.nz * 19 * sizeof(double));
    L.outw = take((size_t)gr.ny * gr.nz * sizeof(double));  // characteristic outlet
    L.total = off;
    return L;
}

// Fixed-order reduction of the partial slots: ntile step tiles, then nisl
// island workgroups, then nmlp surrogate slots.  The island's sums and extrema
// describe the last step only if it listed cells (*count > 0), the
// surrogate's only if the last step ran it (mlp_live); counters always
// accumulate.
__global__ void reduce_partials(const double* __restrict__ part, int ntile, int nisl, int nmlp,
                                int ns, double* __restrict__ out,
                                const int* __restrict__ count, int mlp_live) {
    const bool island_live = count != nullptr && *count > 0;
    const int nblocks = ntile + nisl + nmlp;
    __shared__ double sh[BLOCK];
    const int t = threadIdx.x;
    for (int s = 0; s < DG_COUNT; ++s) {
        if (s >= DG_SP + ns && s < DG_ENTH) {
            if (t == 0) out[s] = 0.0;
            continue;
        }
        const bool mx = s == DG_UMAX || s == DG_TMAX, mn = s == DG_TMIN;
        double acc = mx ? -1e300 : mn ? 1e300 : 0.0;
        const bool cnt = s >= DG_NONFIN;
        for (int b = t; b < nblocks; b += BLOCK) {
            if (!(b < ntile || cnt || (b < ntile + nisl ? island_live : mlp_live != 0))) continue;
            const double v = part[(size_t)b * DIAG_STRIDE + s];
            acc = mx ? fmax(acc, v) : mn ? fmin(acc, v) : acc + v;
        }
        sh[t] = acc;
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (t < w) {
                const double v = sh[t + w];
                sh[t] = mx ? fmax(sh[t], v) : mn ? fmin(sh[t], v) : sh[t] + v;
            }
            __syncthreads();
        }
        if (t == 0) out[s] = sh[0];
        __syncthreads();
    }
}

// Closed domain: P0 / P0_in from the sum S of M / T over the cells (mode 0:
// the initial state, from the P0 sum kernel's (sum, compensation) pairs, p = 1;
// mode 1: after a step, from the per-slot sums the step's kernels wrote -- the
// tiles, the island's workgroups if it listed cells, the surrogate's slots if
// the step ran it --, p = S0 / S; mode
// 2: no new sum), then the parameter blocks' EOS numerator and the step's
// dP0/dt terms for the next step.  The slot sums are combined in a fixed order
// with compensation (Neumaier), eight loads in flight per thread.
constexpr int P0_THREADS = 1024;
__global__ __launch_bounds__(P0_THREADS) void p0_update_kernel(
    const double* __restrict__ part, const double* __restrict__ mt, int ntile, int nisl,
    int nmlp, const int* __restrict__ count, int mlp_live, P0State* __restrict__ st,
    Par<float>* __restrict__ pf, Par<double>* __restrict__ pd, int mode) {
    __shared__ double sh[P0_THREADS], shc[P0_THREADS];
    const int t = threadIdx.x;
    double acc = 0.0, cmp = 0.0;  // compensated, as the partial sums
    auto add = [](double& s, double& c, double x) {
        const double u = s + x;
        c += fabs(s) >= fabs(x) ? (s - u) + x : (x - u) + s;
        s = u;
    };
    if (mode == 0) {
        for (int i = t; i < P0_PARTS; i += P0_THREADS) {
            cmp += part[2 * i + 1];
            add(acc, cmp, part[2 * i]);
        }
    } else if (mode == 1) {
        const bool island_live = count != nullptr && *count > 0;
        const int n = ntile + nisl + nmlp;
        for (int i0 = t; i0 < n; i0 += 8 * P0_THREADS) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u * P0_THREADS;
                const bool use = i < ntile || (i < ntile + nisl ? island_live : mlp_live != 0);
                v[u] = i < n && use ? mt[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) add(acc, cmp, v[u]);
        }
    }
    sh[t] = acc;
    shc[t] = cmp;
    __syncthreads();
    for (int o = P0_THREADS / 2; o > 0; o >>= 1) {
        if (t < o) {
            double s = sh[t], c = shc[t] + shc[t + o];
            add(s, c, sh[t + o]);
            sh[t] = s;
            shc[t] = c;
        }
        __syncthreads();
    }
    if (t == 0) {
        P0State q = *st;
        const double S = sh[0] + shc[0];
        if (mode == 0) {
            q.S0 = S;
            q.p = q.p_prev = 1.0;
        } else if (mode == 1) {
            q.p_prev = q.p;
            q.p = q.S0 / S;
        }
        *st = q;
        const double dp = q.p - q.p_prev, rr = q.rho_ref0 * q.p, dt = q.P0_in * dp, dl = dp / q.p;
        pd->rho_ref = rr;
        pd->p0 = q.p;
        pd->dp0_term = dt;
        pd->dlnp0 = dl;
        pf->rho_ref = (float)rr;
        pf->p0 = (float)q.p;
        pf->dp0_term = (float)dt;
        pf->dlnp0 = (float)dl;
    }
}

}  // namespace

struct lbfd_ctx {
    lbfd_grid grid;
    Layout L;
    int dim, Q, ns, nsm;
    size_t N;
    bool fp32;
    int device;
    hipStream_t stream;
    char* ws;
    lbfd_params params;
    HostMech mech;
    bool have_phi = false, have_params = false, have_mech = false, have_state = false;
    int cur = 0, odd = 0;
    bool last_sur = false;  // the last step ran the surrogate (its diagnostics slots are live)
    int mlp_grid = 0;       // surrogate workgroups (two diagnostics slots each)
    double state_T[2] = {0.0, 0.0};  // min and max T of the initial state
    double T_ref = 0.0;  // the temperature planes hold T - T_ref (FP32: T_solid at init_state)
    int64_t steps = 0;
    std::string err;
    // launch timing: event pairs per kernel kind, reused across enable cycles
    bool timing = false;
    std::vector<hipEvent_t> ev[3];
    size_t ev_used[3] = {0, 0, 0};
    // chemistry surrogate
    bool sur = false;
    int n_cu = 0;
    // sharp-interface mode: solid flags of the phase field (phi >= 1/2, FP64
    // decision), uploaded with it; the link masks are rebuilt on the device
    // before the next step or read after the flags changed
    std::vector<uint8_t> solid;
    bool mask_dirty = true;
    // velocity inlet profile [dim][ny*nz] (empty: the uniform u_in)
    std::vector<double> prof;
};

namespace {

lbfd_status fail(lbfd_ctx* c, lbfd_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

lbfd_status hip_check(lbfd_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return LBFD_OK;
    return fail(c, LBFD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
T* dptr(lbfd_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

// Wilke interaction coefficient Phi_kj of the mixture viscosity rule.
double wilke(double muk, double muj, double Mk, double Mj) {
    const double a = 1.0 + std::sqrt((muk / muj) * std::sqrt(Mj / Mk));
    return a * a / (std::sqrt(8.0) * std::sqrt(1.0 + Mk / Mj));
}

// Validated host copy of a mechanism table.
lbfd_status mech_from_abi(const lbfd_mechanism* m, HostMech& h, std::string& msg) {
    if (m->n_reactions < 0 || m->n_reactions > LBFD_MAX_REACTIONS)
        return msg = "n_reactions out of range", LBFD_E_INVAL;
    const int ns = m->n_species, nr = m->n_reactions;
    if (ns < 0 || ns > LBFD_MAX_SPECIES) return msg = "n_species out of range", LBFD_E_INVAL;
    if (ns > 0 && (!m->M || !m->dhf || !m->mu_star)) return msg = "null table", LBFD_E_INVAL;
    if (nr > 0 && (!m->nu_f || !m->nu_r || !m->A || !m->beta || !m->theta || !m->reversible ||
                   !m->lnKc_a || !m->lnKc_b))
        return msg = "null table", LBFD_E_INVAL;
    h = HostMech();
    h.ns = ns;
    h.nr = nr;
    for (int k = 0; k < ns; ++k) {
        if (!(m->M[k] > 0.0) || !(m->mu_star[k] > 0.0) || !std::isfinite(m->dhf[k]) ||
            !std::isfinite(m->M[k]) || !std::isfinite(m->mu_star[k]))
            return msg = "bad species data", LBFD_E_INVAL;
        h.M.push_back(m->M[k]);
        h.dhf.push_back(m->dhf[k]);
        h.mu_star.push_back(m->mu_star[k]);
        if (m->cp) {
            if (!(m->cp[k] > 0.0) || !std::isfinite(m->cp[k]))
                return msg = "species heat capacities must be positive", LBFD_E_INVAL;
            h.cp.push_back(m->cp[k]);
        }
    }
    for (int j = 0; j < nr; ++j) {
        if (!(m->A[j] >= 0.0) || !std::isfinite(m->A[j]) || !std::isfinite(m->beta[j]) ||
            !std::isfinite(m->theta[j]) || !std::isfinite(m->lnKc_a[j]) ||
            !std::isfinite(m->lnKc_b[j]))
            return msg = "bad rate data", LBFD_E_INVAL;
        h.A.push_back(m->A[j]);
        h.beta.push_back(m->beta[j]);
        h.theta.push_back(m->theta[j]);
        h.lnKc_a.push_back(m->lnKc_a[j]);
        h.lnKc_b.push_back(m->lnKc_b[j]);
        h.rev.push_back(m->reversible[j] ? 1 : 0);
        int order_f = 0, order_r = 0;
        for (int k = 0; k < ns; ++k) {
            const int f = m->nu_f[j * ns + k], r = m->nu_r[j * ns + k];
            if (f < 0 || f > 3 || r < 0 || r > 3)
                return msg = "stoichiometric coefficients must be 0..3", LBFD_E_INVAL;
            h.nu_f.push_back(f);
            h.nu_r.push_back(r);
            order_f += f;
            order_r += r;
        }
        if (order_f > 4 || order_r > 4) return msg = "reaction order of a side above 4", LBFD_E_INVAL;
    }
    return LBFD_OK;
}

// ------------------------------------------------------ stability rule
// Host closures of the check (the same definitions as the kernels' closures,
// in FP64): Sutherland ratio, and viscosity / conductivity of one state.
double host_sutherland(const lbfd_params& p, double T) {
    if (p.mu_model == 0) return 1.0;
    const double x = T / p.T_in;
    return x * std::sqrt(x) * (p.T_in + p.sutherland_S) / (T + p.sutherland_S);
}
void host_transport(const lbfd_params& p, int ns, const HostMech* m, double T, const double* Y,
                    double& mu, double& lam) {
    const double mu0 = p.rho_in * p.nu_in * host_sutherland(p, T);
    if (p.transport_model == 1 && ns > 0 && m) {
        double im = 0.0, X[LBFD_MAX_SPECIES];
        for (int k = 0; k < ns; ++k) im += Y[k] / m->M[k];
        for (int k = 0; k < ns; ++k) X[k] = Y[k] / (m->M[k] * im);
        double mm = 0.0, l1 = 0.0, l2 = 0.0;
        for (int k = 0; k < ns; ++k) {
            double den = 0.0;
            for (int j = 0; j < ns; ++j)
                den += wilke(m->mu_star[k], m->mu_star[j], m->M[k], m->M[j]) * X[j];
            const double muk = m->mu_star[k] * mu0, lk = muk * p.cp / p.Pr;
            if (X[k] > 0.0) mm += muk * X[k] / den;
            l1 += X[k] * lk;
            l2 += X[k] / lk;
        }
        mu = mm;
        lam = 0.5 * (l1 + 1.0 / l2);
        return;
    }
    mu = mu0;
    lam = mu0 * p.cp / p.Pr;
}

// The rule of lbfd_stability over [min(T_lo, given temperatures), max(T_hi, ...)].
lbfd_status stability_eval(const lbfd_grid& g, const lbfd_params& p, const HostMech* m,
                           double T_lo, double T_hi, lbfd_stability_report& r, std::string& msg) {
    std::memset(&r, 0, sizeof(r));
    const int ns = g.n_species, d = g.dim;
    double lo = p.T_in, hi = p.T_in;
    auto take = [&](double t) {
        if (t > 0.0 && std::isfinite(t)) {
            lo = std::min(lo, t);
            hi = std::max(hi, t);
        }
    };
    take(p.T_solid);
    take(p.T_max);
    for (int f = 0; f < 6; ++f)
        if (g.fd_bc[f] == LBFD_FD_DIRICHLET) take(p.fd_face[f][0]);
    take(T_lo);
    take(T_hi);
    r.T_lo = lo;
    r.T_hi = hi;
    // density of the inlet mixture (its molar mass is the EOS reference, so
    // rho = rho_in T_in / T); viscosity and conductivity of the closure
    double Y[LBFD_MAX_SPECIES];
    for (int k = 0; k < ns; ++k) Y[k] = p.Y_in[k];
    double mu, lam;
    host_transport(p, ns, m, lo, Y, mu, lam);
    const double rho_lo = p.rho_in * p.T_in / lo;
    r.tau_lo = mu / (rho_lo / 3.0) + 0.5;
    host_transport(p, ns, m, hi, Y, mu, lam);
    const double rho_hi = p.rho_in * p.T_in / hi;
    r.alpha_hi = lam / (rho_hi * p.cp);
    double le_min = 1.0;
    for (int k = 0; k < ns; ++k) le_min = std::min(le_min, p.Le[k]);
    r.D_hi = ns > 0 ? r.alpha_hi / le_min : 0.0;
    r.h_hi = p.A_T * r.alpha_hi * (4.0 / 27.0) / (p.eta * p.eta);
    r.u_sum = std::sqrt((double)d) * 0.1;
    r.fd_sum = 2.0 * d * std::max(r.alpha_hi, r.D_hi) + r.h_hi + r.u_sum;
    // pseudo-first-order consumption rate of each species at T_hi
    if (m && ns > 0 && m->nr > 0) {
        double X[LBFD_MAX_SPECIES], kap[LBFD_MAX_SPECIES] = {0.0};
        for (int k = 0; k < ns; ++k) X[k] = rho_hi * std::max(p.Y_in[k], 0.01) / m->M[k];
        for (int j = 0; j < m->nr; ++j) {
            const double lkf =
                std::log(std::max(m->A[j], 1e-300)) + m->beta[j] * std::log(hi) - m->theta[j] / hi;
            for (int side = 0; side < (m->rev[j] ? 2 : 1); ++side) {
                const int* nu = side == 0 ? &m->nu_f[j * ns] : &m->nu_r[j * ns];
                const double lk = side == 0 ? lkf : lkf - (m->lnKc_a[j] + m->lnKc_b[j] / hi);
                if (m->A[j] == 0.0) continue;
                for (int k = 0; k < ns; ++k) {
                    if (nu[k] == 0) continue;
                    double v = nu[k] * std::exp(lk);
                    for (int q = 0; q < ns; ++q) v *= std::pow(X[q], nu[q] - (q == k ? 1 : 0));
                    kap[k] += v;
                }
            }
        }
        for (int k = 0; k < ns; ++k) r.kappa_hi = std::max(r.kappa_hi, kap[k]);
        r.h_kappa = r.kappa_hi / p.n_sub;
    }
    if (!std::isfinite(r.tau_lo) || !std::isfinite(r.fd_sum) || !std::isfinite(r.h_kappa))
        r.violated |= 8;
    if (!(r.tau_lo > 0.5 + 1e-3)) r.violated |= 1;
    if (!(r.fd_sum <= 0.9)) r.violated |= 2;
    // the linearly implicit scheme is stable at any h kappa: no reaction bound
    if (!(r.h_kappa <= 0.5) && p.chem_scheme != 1) r.violated |= 4;
    if (!r.violated) return LBFD_OK;
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "explicit stability over %.1f..%.1f K: tau(T_lo) = %.4g (> 0.501), "
                  "2 dim max(alpha, D) + H/(rho cp) + sum|u| = %.4g (<= 0.9; alpha %.4g, D %.4g, "
                  "H/(rho cp) %.4g, sum|u| %.4g), kappa/n_sub = %.4g (<= 0.5)",
                  lo, hi, r.tau_lo, r.fd_sum, r.alpha_hi, r.D_hi, r.h_hi, r.u_sum, r.h_kappa);
    msg = buf;
    return LBFD_E_INVAL;
}

template <typename R>
Par<R> build_par(const lbfd_ctx* c) {
    Par<R> P;
    std::memset(&P, 0, sizeof(P));
    const lbfd_params& p = c->params;
    const lbfd_grid& g = c->grid;
    P.nx = g.nx;
    P.ny = g.ny;
    P.nz = g.nz;
    P.ns = c->ns;
    P.nr = c->ns > 0 ? c->mech.nr : 0;
    P.n_sub = p.n_sub;
    P.chem_scheme = p.chem_scheme;
    P.mu_model = p.mu_model;
    P.transport = p.transport_model;
    // temperature planes hold T - T_ref (FP32 mode: T_solid of the params the
    // state was initialised with; FP64 mode: 0)
    const double T_ref = c->T_ref;
    P.T_ref = (R)T_ref;
    P.Ts_rel = (R)(p.T_solid - T_ref);
    for (int f = 0; f < 6; ++f) {
        P.lb_bc[f] = g.lb_bc[f];
        P.fd_bc[f] = g.fd_bc[f];
        P.fd_face[f][0] = (R)(p.fd_face[f][0] - T_ref);
        for (int k = 1; k <= c->ns; ++k) P.fd_face[f][k] = (R)p.fd_face[f][k];
    }
    P.A_u = (R)p.A_u;
    P.A_T = (R)p.A_T;
    P.inv_eta2 = (R)(1.0 / (p.eta * p.eta));
    P.T_s = (R)p.T_solid;
    P.cp = (R)p.cp;
    P.inv_cp = (R)(1.0 / p.cp);
    P.inv_Pr = (R)(1.0 / p.Pr);
    P.rho_in = (R)p.rho_in;
    P.T_in = (R)p.T_in;
    P.inv_T_in = (R)(1.0 / p.T_in);
    P.p0 = (R)1;  // a closed domain's P0 ratio is written on the device
    P.mu_ref = (R)(p.rho_in * p.nu_in);
    P.S = (R)p.sutherland_S;
    P.S_T_in = (R)(p.T_in + p.sutherland_S);
    P.theta_ign = (R)p.ign_threshold;
    P.h_sub = (R)(1.0 / p.n_sub);
    for (int a = 0; a < 3; ++a) {
        P.u_in[a] = (R)(a < c->dim ? p.u_in[a] : 0.0);
        P.F_b[a] = (R)(a < c->dim ? p.body_force[a] : 0.0);
    }
    {
        const double u0 = p.u_in[0], u1 = c->dim > 1 ? p.u_in[1] : 0.0,
                     u2 = c->dim > 2 ? p.u_in[2] : 0.0;
        const double uu = u0 * u0 + u1 * u1 + u2 * u2;
        for (int j = 0; j < c->Q; ++j) {
            const int* cx = c->dim == 2 ? Lat<2>::cx : Lat<3>::cx;
            const int* cy = c->dim == 2 ? Lat<2>::cy : Lat<3>::cy;
            const int* cz = c->dim == 2 ? Lat<2>::cz : Lat<3>::cz;
            const double cu = cx[j] * u0 + cy[j] * u1 + cz[j] * u2;
            const double e = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
            P.inlet_eq[j] = (R)(p.rho_in * (1.0 / 3.0) * e);
        }
    }
    {  // characteristic outlet: K = sigma c_s (1 - Ma^2) / nx, Ma = |u_in| / c_s
        const double cs = std::sqrt(1.0 / 3.0);
        const double uin2 = p.u_in[0] * p.u_in[0] + p.u_in[1] * p.u_in[1] + p.u_in[2] * p.u_in[2];
        P.char_out = g.lb_bc[1] == LBFD_LB_CHARACTERISTIC_OUTLET;
        P.K_out = (R)(p.outlet_sigma * cs * (1.0 - uin2 / (1.0 / 3.0)) / g.nx);
        P.c_s = (R)cs;
    }
    double im_in = 0.0;
    int corr = 0;
    for (int k = 0; k < c->ns; ++k) {
        // with species heat capacities rho D_k = (lambda / c_p) / Le_k, the
        // mixture c_p taken per cell
        P.rD_fac[k] = c->mech.cp.empty() ? (R)(1.0 / (p.cp * p.Le[k])) : (R)(1.0 / p.Le[k]);
        P.cp_k[k] = c->mech.cp.empty() ? (R)p.cp : (R)c->mech.cp[k];
        if (p.Le[k] != p.Le[0]) corr = 1;
        P.M[k] = (R)c->mech.M[k];
        P.invM[k] = (R)(1.0 / c->mech.M[k]);
        P.dhf[k] = (R)c->mech.dhf[k];
        P.mu_star[k] = (R)c->mech.mu_star[k];
        im_in += p.Y_in[k] / c->mech.M[k];
    }
    P.corr = corr;
    P.cpk = c->ns > 0 && !c->mech.cp.empty();
    P.any_beta = 0;
    for (int j = 0; j < P.nr; ++j)
        if (c->mech.beta[j] != 0.0) P.any_beta = 1;
    P.rho_ref = c->ns > 0 ? (R)(p.rho_in * p.T_in / (1.0 / im_in)) : (R)(p.rho_in * p.T_in);
    for (int k = 0; k < c->ns; ++k)
        for (int j = 0; j < c->ns; ++j)
            P.Phi[k][j] =
                (R)wilke(c->mech.mu_star[k], c->mech.mu_star[j], c->mech.M[k], c->mech.M[j]);
    // padding species: mu* = 1 and a row of ones in Phi (denominator
    // sum X = 1), so that their X = 0 adds exact zeros to the Wilke sums
    for (int k = c->ns; k < MAXS; ++k) {
        P.mu_star[k] = (R)1;
        for (int j = 0; j < MAXS; ++j) P.Phi[k][j] = (R)1;
    }
    for (int k = 0; k < MAXS; ++k)
        P.inv_mu_star[k] = k < c->ns ? (R)(1.0 / c->mech.mu_star[k]) : (R)1;
    P.Pr_over_cp = (R)(p.Pr / p.cp);
    // The reaction table: reactions whose sides have at most two factors
    // first, then the others, each segment in the mechanism's order and
    // padded to the kernel's reaction group; index words pad with the
    // kernel's species bound (its concentration slot holds 1).
    const int nsm = nsm_bucket(c->ns);
    const uint32_t pad = (uint32_t)nsm;
    const int group = nsm >= 9 ? 2 : 1;
    Rxn<R>& x = P.rx;
    for (int j = 0; j < MAXR_TAB; ++j) x.fidx[j] = x.ridx[j] = pad * 0x01010101u;
    int e = 0;
    for (int seg = 0; seg < 2; ++seg) {
        for (int j = 0; j < P.nr; ++j) {
            int of = 0, orr = 0;
            for (int k = 0; k < c->ns; ++k) {
                of += c->mech.nu_f[j * c->ns + k];
                orr += c->mech.nu_r[j * c->ns + k];
            }
            if ((of <= 2 && orr <= 2) != (seg == 0)) continue;
            // FP32: exponents in base 2 (theta and ln K_c scaled by log2 e)
            const double l2e = sizeof(R) == 4 ? 1.4426950408889634 : 1.0;
            x.A[e] = (R)c->mech.A[j];
            x.beta[e] = (R)c->mech.beta[j];
            x.theta[e] = (R)(c->mech.theta[j] * l2e);
            x.rev[e] = c->mech.rev[j];
            if (x.rev[e]) {
                x.lnKc_a[e] = (R)(c->mech.lnKc_a[j] * l2e);
                x.lnKc_b[e] = (R)(c->mech.lnKc_b[j] * l2e);
            } else {
                x.lnKc_a[e] = std::numeric_limits<R>::infinity();  // reverse term exactly 0
            }
            uint32_t fw = 0, rw = 0;
            int nf = 0, nr = 0;
            for (int k = 0; k < c->ns; ++k) {
                const int f = c->mech.nu_f[j * c->ns + k], r = c->mech.nu_r[j * c->ns + k];
                for (int q = 0; q < f; ++q) fw |= (uint32_t)k << (8 * nf++);
                for (int q = 0; q < r; ++q) rw |= (uint32_t)k << (8 * nr++);
                x.nud[e][k] = (R)(r - f);
            }
            for (; nf < 4; ++nf) fw |= pad << (8 * nf);
            for (; nr < 4; ++nr) rw |= pad << (8 * nr);
            x.fidx[e] = fw;
            x.ridx[e] = rw;
            ++e;
        }
        e = (e + group - 1) / group * group;  // inert padding (zeroed, A = 0)
        if (seg == 0) P.n_lo = e;
    }
    P.n_tab = e;
    return P;
}

bool ready_for_tables(const lbfd_ctx* c) { return c->have_params && (c->ns == 0 || c->have_mech); }

// The stability rule for a context with the given params and mechanism, over
// the temperatures of the initial state when one was set.
// Extended boundaries of a grid: the characteristic outlet, or an FD
// Dirichlet face on an LB-periodic axis.
bool grid_ext(const lbfd_grid& g) {
    if (g.lb_bc[1] == LBFD_LB_CHARACTERISTIC_OUTLET) return true;
    for (int f = 0; f < 6; ++f)
        if (g.lb_bc[f] == LBFD_LB_PERIODIC && g.fd_bc[f] != LBFD_FD_PERIODIC) return true;
    return false;
}

// The step runs the kernels of the extended boundaries (sharp-interface
// masks, inlet profile, characteristic outlet, thermal walls on periodic
// axes); they exist for up to four species.
bool uses_ext(const lbfd_ctx* c) {
    return c->params.sharp_interface || !c->prof.empty() || grid_ext(c->grid);
}

lbfd_status check_stable(lbfd_ctx* c, const lbfd_params& p, const HostMech* m) {
    if (m && !m->cp.empty()) {  // what the kernels with species heat capacities cover
        if (p.transport_model != 0)
            return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: single-gas transport only");
        if (p.chem_scheme != 0)
            return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: explicit reaction scheme only");
        if (p.sharp_interface)
            return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: no sharp-interface mode");
        if (c->nsm > 9)
            return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: at most 9 species");
        if (c->sur)
            return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: no surrogate");
        if (grid_ext(c->grid) || !c->prof.empty())
            return fail(c, LBFD_E_UNSUPPORTED,
                        "species heat capacities: no characteristic outlet, inlet profile or "
                        "thermal walls on periodic axes");
        if (p.closed)
            for (double v : m->cp)
                if (!(p.r_gas < v))
                    return fail(c, LBFD_E_INVAL, "closed domain: r_gas below every c_p,k");
    }
    lbfd_stability_report r;
    std::string msg;
    const lbfd_status st = stability_eval(c->grid, p, m, c->have_state ? c->state_T[0] : 0.0,
                                          c->have_state ? c->state_T[1] : 0.0, r, msg);
    return st ? fail(c, st, msg) : LBFD_OK;
}

// Closed domain: the P0 update (mode as in p0_update_kernel), on the context's
// stream; the initial state's sum of M / T comes from the P0 sum kernel, a
// step's from the slots its kernels filled (StepArgs::mt).
lbfd_status launch_p0(lbfd_ctx* c, int mode) {
    hipError_t e = hipSuccess;
    double* part = dptr<double>(c, c->L.p0part);
    if (mode == 0) {
        const int N = (int)c->N;
        if (c->fp32)
            e = launch_p0_sum_f32(dptr<float>(c, c->cur ? c->L.T1 : c->L.T0),
                                  dptr<float>(c, c->cur ? c->L.Y1 : c->L.Y0), N, c->ns,
                                  dptr<Par<float>>(c, c->L.parf), part, c->stream);
        else
            e = launch_p0_sum_f64(dptr<double>(c, c->cur ? c->L.T1 : c->L.T0),
                                  dptr<double>(c, c->cur ? c->L.Y1 : c->L.Y0), N, c->ns,
                                  dptr<Par<double>>(c, c->L.pard), part, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "P0 sum");
    }
    // the island's and the surrogate's slots exist in FP32 mode with species
    const bool island = c->fp32 && c->ns > 0;
    hipLaunchKernelGGL(p0_update_kernel, dim3(1), dim3(P0_THREADS), 0, c->stream, part,
                       dptr<double>(c, c->L.mtpart), c->L.nblocks, island ? ISLAND_WG : 0,
                       island ? 2 * c->mlp_grid : 0, island ? dptr<int>(c, c->L.count) : nullptr,
                       c->last_sur ? 1 : 0, dptr<P0State>(c, c->L.p0),
                       dptr<Par<float>>(c, c->L.parf), dptr<Par<double>>(c, c->L.pard), mode);
    return hip_check(c, hipGetLastError(), "P0 update");
}

lbfd_status upload_tables(lbfd_ctx* c) {
    if (!ready_for_tables(c)) return LBFD_OK;
    Par<double> pd = build_par<double>(c);
    Par<float> pf = build_par<float>(c);
    lbfd_status st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.pard), &pd, sizeof(pd),
                                                 hipMemcpyHostToDevice, c->stream),
                               "upload parameters");
    if (st) return st;
    st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.parf), &pf, sizeof(pf),
                                     hipMemcpyHostToDevice, c->stream),
                   "upload parameters");
    if (st) return st;
    if (!c->prof.empty()) {  // per-row inlet equilibria rho_in c_s^2 e_j(u(y, z))
        const size_t nr = (size_t)c->grid.ny * c->grid.nz;
        std::vector<double> eq(nr * 19, 0.0);
        const int* cx = c->dim == 2 ? Lat<2>::cx : Lat<3>::cx;
        const int* cy = c->dim == 2 ? Lat<2>::cy : Lat<3>::cy;
        const int* cz = c->dim == 2 ? Lat<2>::cz : Lat<3>::cz;
        for (size_t r = 0; r < nr; ++r) {
            const double u0 = c->prof[r], u1 = c->prof[nr + r],
                         u2 = c->dim > 2 ? c->prof[2 * nr + r] : 0.0;
            const double uu = u0 * u0 + u1 * u1 + u2 * u2;
            for (int j = 0; j < c->Q; ++j) {
                const double cu = cx[j] * u0 + cy[j] * u1 + cz[j] * u2;
                eq[r * 19 + j] = c->params.rho_in * (1.0 / 3.0) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            }
        }
        st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.inlet), eq.data(), eq.size() * 8,
                                         hipMemcpyHostToDevice, c->stream),
                       "upload inlet profile");
        if (st) return st;
        st = hip_check(c, hipStreamSynchronize(c->stream), "upload inlet profile");
        if (st) return st;
    }
    // a closed domain keeps its P0 across new parameters
    if (c->params.closed && c->have_state && (st = launch_p0(c, 2))) return st;
    return hip_check(c, hipStreamSynchronize(c->stream), "upload parameters");
}

// host FP64 -> device field of the context's precision (minus `shift`,
// applied in FP64 before the rounding: the temperature planes)
lbfd_status upload_field(lbfd_ctx* c, size_t off, const double* src, size_t n,
                         double shift = 0.0, double scale = 1.0) {
    if (scale != 1.0) {  // stored as scale * value (the populations)
        std::vector<double> tmp(n);
        for (size_t i = 0; i < n; ++i) tmp[i] = src[i] * scale;
        return upload_field(c, off, tmp.data(), n, shift, 1.0);
    }
    if (c->fp32) {
        std::vector<float> tmp(n);
        for (size_t i = 0; i < n; ++i) tmp[i] = (float)(src[i] - shift);
        lbfd_status st = hip_check(
            c, hipMemcpyAsync(dptr<char>(c, off), tmp.data(), n * 4, hipMemcpyHostToDevice, c->stream),
            "upload");
        if (st) return st;
        return hip_check(c, hipStreamSynchronize(c->stream), "upload");
    }
    lbfd_status st = hip_check(
        c, hipMemcpyAsync(dptr<char>(c, off), src, n * 8, hipMemcpyHostToDevice, c->stream), "upload");
    if (st) return st;
    return hip_check(c, hipStreamSynchronize(c->stream), "upload");
}

lbfd_status download_field(lbfd_ctx* c, size_t off, double* dst, size_t n, double shift = 0.0,
                           double scale = 1.0) {
    if (scale != 1.0) {
        lbfd_status st = download_field(c, off, dst, n, shift, 1.0);
        if (st) return st;
        for (size_t i = 0; i < n; ++i) dst[i] /= scale;
        return LBFD_OK;
    }
    if (c->fp32) {
        std::vector<float> tmp(n);
        lbfd_status st = hip_check(
            c, hipMemcpyAsync(tmp.data(), dptr<char>(c, off), n * 4, hipMemcpyDeviceToHost, c->stream),
            "download");
        if (st) return st;
        st = hip_check(c, hipStreamSynchronize(c->stream), "download");
        if (st) return st;
        for (size_t i = 0; i < n; ++i) dst[i] = (double)tmp[i] + shift;
        return LBFD_OK;
    }
    lbfd_status st = hip_check(
        c, hipMemcpyAsync(dst, dptr<char>(c, off), n * 8, hipMemcpyDeviceToHost, c->stream), "download");
    if (st) return st;
    return hip_check(c, hipStreamSynchronize(c->stream), "download");
}

size_t elem(const lbfd_ctx* c) { return c->fp32 ? 4 : 8; }
// stored populations = scale * g (FP32: 36, so that the weights are integers)
double pop_scale(const lbfd_ctx* c) { return c->fp32 ? Pop<float>::scale : Pop<double>::scale; }

lbfd_status validate_grid(const lbfd_grid* g, std::string& msg) {
    if (!g) return msg = "null grid", LBFD_E_INVAL;
    if (g->dim != 2 && g->dim != 3) return msg = "dim must be 2 or 3", LBFD_E_INVAL;
    if (g->nx < 2 || g->ny < 1 || g->nz < 1) return msg = "grid too small", LBFD_E_INVAL;
    if (g->dim == 2 && g->nz != 1) return msg = "dim 2 needs nz == 1", LBFD_E_INVAL;
    if (g->precision != LBFD_FP32 && g->precision != LBFD_FP64)
        return msg = "unknown precision", LBFD_E_INVAL;
    if (g->n_species < 0 || g->n_species > LBFD_MAX_SPECIES)
        return msg = "n_species out of range", LBFD_E_INVAL;
    const double N = (double)g->nx * g->ny * g->nz;
    if (N * lattice_q(g->dim) > (double)INT_MAX) return msg = "grid too large", LBFD_E_INVAL;
    const int nf = g->dim == 2 ? 4 : 6;
    for (int f = 0; f < 6; ++f) {
        const int lb = g->lb_bc[f], fd = g->fd_bc[f];
        if (lb < 0 || lb > 4 || fd < 0 || fd > 2) return msg = "unknown boundary kind", LBFD_E_INVAL;
        if (f >= nf && (lb != LBFD_LB_PERIODIC || fd != LBFD_FD_PERIODIC))
            return msg = "z faces of a 2-D grid must be periodic", LBFD_E_INVAL;
        if (fd == LBFD_FD_PERIODIC && lb != LBFD_LB_PERIODIC)
            return msg = "an FD-periodic face needs an LB-periodic one", LBFD_E_INVAL;
        if (lb == LBFD_LB_PERIODIC && fd == LBFD_FD_ZERO_GRADIENT)
            return msg = "an LB-periodic face takes a periodic or Dirichlet FD kind",
                   LBFD_E_INVAL;
        if (nsm_bucket(g->n_species) > 4 &&
            (lb == LBFD_LB_CHARACTERISTIC_OUTLET ||
             (lb == LBFD_LB_PERIODIC && fd != LBFD_FD_PERIODIC)))
            return msg = "characteristic outlet and thermal walls on periodic axes: at most 4 "
                         "species", LBFD_E_UNSUPPORTED;
        if (lb == LBFD_LB_VELOCITY_INLET && f != 0)
            return msg = "velocity inlet only on the -x face", LBFD_E_UNSUPPORTED;
        if ((lb == LBFD_LB_PRESSURE_OUTLET || lb == LBFD_LB_CHARACTERISTIC_OUTLET) && f != 1)
            return msg = "pressure outlet only on the +x face", LBFD_E_UNSUPPORTED;
    }
    for (int a = 0; a < 3; ++a)
        if ((g->lb_bc[2 * a] == LBFD_LB_PERIODIC) != (g->lb_bc[2 * a + 1] == LBFD_LB_PERIODIC))
            return msg = "both faces of an axis must be periodic or neither", LBFD_E_INVAL;
    return LBFD_OK;
}

// Record the start (end = false) or end event of a timed launch of `kernel`.
hipError_t time_mark(lbfd_ctx* c, int kernel, bool end) {
    if (!c->timing) return hipSuccess;
    std::vector<hipEvent_t>& v = c->ev[kernel];
    size_t& used = c->ev_used[kernel];
    const size_t slot = end ? used - 1 : used;
    if (!end) {
        if (2 * used + 2 > v.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                v.push_back(e);
            }
        }
        ++used;
    }
    return hipEventRecord(v[2 * slot + (end ? 1 : 0)], c->stream);
}

// Sharp-interface mode: link masks from the solid flags, when they changed
lbfd_status ensure_si_mask(lbfd_ctx* c) {
    if (!c->params.sharp_interface || !c->mask_dirty) return LBFD_OK;
    hipError_t e;
    if (c->fp32)
        e = launch_si_mask_f32(c->dim, dptr<uint8_t>(c, c->L.solid),
                               dptr<Par<float>>(c, c->L.parf), dptr<uint32_t>(c, c->L.smask),
                               (int)c->N, c->stream);
    else
        e = launch_si_mask_f64(c->dim, dptr<uint8_t>(c, c->L.solid),
                               dptr<Par<double>>(c, c->L.pard), dptr<uint32_t>(c, c->L.smask),
                               (int)c->N, c->stream);
    lbfd_status st = hip_check(c, e, "link mask kernel launch");
    if (st) return st;
    c->mask_dirty = false;
    return LBFD_OK;
}

template <typename R>
lbfd_status launch_step(lbfd_ctx* c, int phase) {
    lbfd_status st = ensure_si_mask(c);
    if (st) return st;
    StepArgs<R> a;
    const size_t N = c->N;
    a.g = dptr<R>(c, c->L.g);
    a.T_cur = dptr<R>(c, c->cur ? c->L.T1 : c->L.T0);
    a.T_nxt = dptr<R>(c, c->cur ? c->L.T0 : c->L.T1);
    a.Y_cur = dptr<R>(c, c->cur ? c->L.Y1 : c->L.Y0);
    a.Y_nxt = dptr<R>(c, c->cur ? c->L.Y0 : c->L.Y1);
    a.divu = dptr<R>(c, c->L.divu);
    a.phi = dptr<R>(c, c->L.phi);
    a.smask = c->params.sharp_interface ? dptr<uint32_t>(c, c->L.smask) : nullptr;
    a.inlet_prof = c->prof.empty() ? nullptr : dptr<double>(c, c->L.inlet);
    a.outlet_w = dptr<double>(c, c->L.outw);
    a.partials = dptr<double>(c, c->L.part);
    a.flags = dptr<unsigned long long>(c, c->L.flags);
    a.P = dptr<Par<R>>(c, sizeof(R) == 4 ? c->L.parf : c->L.pard);
    a.PD = dptr<Par<double>>(c, c->L.pard);
    a.N = (int)N;
    a.nblocks = c->L.nblocks;
    a.nbx = c->L.nbx;
    a.nby = c->L.nby;
    a.zc = c->L.zc;
    a.odd = c->odd;
    a.phase = phase;
    a.diag = 1;
    a.mtpart = c->params.closed ? dptr<double>(c, c->L.mtpart) : nullptr;
    a.sur = sizeof(R) == 4 && c->sur && c->ns > 0 && c->mech.nr > 0 && (phase & PH_CHEM);
    a.stiff = c->params.chem_scheme;  // 0 none, 1 or 2
    a.cpk = c->ns > 0 && !c->mech.cp.empty();
    a.ext = uses_ext(c);
    a.gtot = dptr<int>(c, c->L.gtot);
    a.list = dptr<int>(c, c->L.list);
    a.count = dptr<int>(c, c->L.count);
    a.P_nx = c->grid.nx;
    a.P_ny = c->grid.ny;
    for (int i = 0; i < 19; ++i) a.gpl[i] = i < c->Q ? a.g + (size_t)i * N : a.g;
    for (int k = 0; k < MAXS; ++k) {
        const int kk = k < c->nsm ? k : 0;
        a.Ycp[k] = a.Y_cur + (size_t)kk * N;
        a.Ynp[k] = a.Y_nxt + (size_t)kk * N;
    }
    hipError_t e;
    if ((e = time_mark(c, LBFD_KERNEL_STEP, false)) != hipSuccess)
        return hip_check(c, e, "timing event");
    if constexpr (sizeof(R) == 4)
        e = launch_step_f32(c->dim, c->nsm, a, c->L.grid, c->stream);
    else
        e = launch_step_f64(c->dim, c->nsm, a, c->L.grid, c->stream);
    if (e == hipSuccess) e = time_mark(c, LBFD_KERNEL_STEP, true);
    if constexpr (sizeof(R) == 4) {
        if (e == hipSuccess && a.sur) {
            e = time_mark(c, LBFD_KERNEL_SURROGATE, false);
            if (e == hipSuccess)
                e = launch_mlp_step_f32(c->dim, c->nsm, a, dptr<SurWeights>(c, c->L.sw),
                                        dptr<SurPar>(c, c->L.sp),
                                        c->mlp_grid, c->stream);
            if (e == hipSuccess) e = time_mark(c, LBFD_KERNEL_SURROGATE, true);
        }
        // every FP32 step with species runs the island (an empty list when no
        // cell is flagged), so that its diagnostics slots describe this step
        if (e == hipSuccess && c->ns > 0) {
            e = time_mark(c, LBFD_KERNEL_ISLAND, false);
            if (e == hipSuccess) e = launch_island_f32(c->dim, c->nsm, a, c->stream);
            if (e == hipSuccess) e = time_mark(c, LBFD_KERNEL_ISLAND, true);
        }
    }
    c->last_sur = a.sur != 0;
    return hip_check(c, e, "step kernel launch");
}

template <typename R>
lbfd_status launch_macro(lbfd_ctx* c) {
    lbfd_status st = ensure_si_mask(c);
    if (st) return st;
    MacroArgs<R> a;
    const size_t N = c->N;
    a.g = dptr<R>(c, c->L.g);
    a.T = dptr<R>(c, c->cur ? c->L.T1 : c->L.T0);
    a.Y = dptr<R>(c, c->cur ? c->L.Y1 : c->L.Y0);
    a.divu = dptr<R>(c, c->L.divu);
    a.phi = dptr<R>(c, c->L.phi);
    a.smask = c->params.sharp_interface ? dptr<uint32_t>(c, c->L.smask) : nullptr;
    a.out = dptr<double>(c, c->L.scratch);
    a.P = dptr<Par<R>>(c, sizeof(R) == 4 ? c->L.parf : c->L.pard);
    a.PD = dptr<Par<double>>(c, c->L.pard);
    a.N = (int)N;
    a.nblocks = c->L.nlin;
    a.odd = c->odd;
    hipError_t e;
    if constexpr (sizeof(R) == 4)
        e = launch_macro_f32(c->dim, c->nsm, a, c->L.nlin, c->stream);
    else
        e = launch_macro_f64(c->dim, c->nsm, a, c->L.nlin, c->stream);
    return hip_check(c, e, "read kernel launch");
}

template <typename R>
lbfd_status launch_init(lbfd_ctx* c, bool with_u) {
    InitArgs<R> a;
    a.g = dptr<R>(c, c->L.g);
    a.T = dptr<R>(c, c->L.T0);
    a.Y = dptr<R>(c, c->L.Y0);
    a.u = with_u ? dptr<double>(c, c->L.scratch) : nullptr;
    a.divu = dptr<R>(c, c->L.divu);
    a.P = dptr<Par<R>>(c, sizeof(R) == 4 ? c->L.parf : c->L.pard);
    a.N = (int)c->N;
    hipError_t e;
    if constexpr (sizeof(R) == 4)
        e = launch_init_f32(c->dim, c->nsm, a, c->L.nlin, c->stream);
    else
        e = launch_init_f64(c->dim, c->nsm, a, c->L.nlin, c->stream);
    return hip_check(c, e, "init kernel launch");
}

lbfd_status set_device(lbfd_ctx* c) { return hip_check(c, hipSetDevice(c->device), "hipSetDevice"); }

}  // namespace

// ====================================================================== ABI

extern "C" {

lbfd_status lbfd_stability(const lbfd_grid* grid, const lbfd_params* params,
                           const lbfd_mechanism* mech, double T_lo, double T_hi,
                           lbfd_stability_report* out) {
    std::string msg;
    if (!params) return LBFD_E_INVAL;
    lbfd_status st = validate_grid(grid, msg);
    if (st) return st;
    HostMech h;
    if (mech) {
        if (mech->n_species != grid->n_species) return LBFD_E_INVAL;
        if ((st = mech_from_abi(mech, h, msg))) return st;
    }
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(params->eta) || !pos(params->cp) || !pos(params->Pr) || !pos(params->rho_in) ||
        !pos(params->T_in) || !(params->nu_in >= 0.0) || params->n_sub < 1)
        return LBFD_E_INVAL;
    for (int k = 0; k < grid->n_species; ++k)
        if (!pos(params->Le[k])) return LBFD_E_INVAL;
    lbfd_stability_report r;
    st = stability_eval(*grid, *params, mech ? &h : nullptr, T_lo, T_hi, r, msg);
    if (out) *out = r;
    return st;
}

lbfd_status lbfd_workspace_bytes(const lbfd_grid* grid, size_t* bytes) {
    std::string msg;
    lbfd_status st = validate_grid(grid, msg);
    if (st) return st;
    if (!bytes) return LBFD_E_INVAL;
    *bytes = make_layout(*grid).total;
    return LBFD_OK;
}

lbfd_status lbfd_create(const lbfd_grid* grid, void* dev_workspace, size_t bytes, void* hip_stream,
                        lbfd_ctx** out) {
    if (!out) return LBFD_E_INVAL;
    *out = nullptr;
    std::string msg;
    lbfd_status st = validate_grid(grid, msg);
    if (st) return st;
    Layout L = make_layout(*grid);
    if (!dev_workspace) return LBFD_E_INVAL;
    if (bytes < L.total) return LBFD_E_NOMEM;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0) return LBFD_E_INVAL;
    lbfd_ctx* c = new (std::nothrow) lbfd_ctx();
    if (!c) return LBFD_E_NOMEM;
    c->grid = *grid;
    c->L = L;
    c->dim = grid->dim;
    c->Q = lattice_q(grid->dim);
    c->ns = grid->n_species;
    c->nsm = nsm_bucket(c->ns);
    c->N = (size_t)grid->nx * grid->ny * grid->nz;
    c->fp32 = grid->precision == LBFD_FP32;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = reinterpret_cast<char*>(dev_workspace);
    std::memset(&c->params, 0, sizeof(c->params));
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess || c->n_cu <= 0) {
        delete c;
        return LBFD_E_DEVICE;
    }
    c->mlp_grid = std::max(1, std::min({c->n_cu, (c->L.nblocks + 1) / 2, MLP_SLOT_WG}));
    *out = c;
    return LBFD_OK;
}

lbfd_status lbfd_set_phase_field(lbfd_ctx* c, const double* phi) {
    if (!c || !phi) return LBFD_E_INVAL;
    for (size_t i = 0; i < c->N; ++i)
        if (!(phi[i] >= 0.0 && phi[i] <= 1.0))
            return fail(c, LBFD_E_INVAL, "phase field outside [0, 1]");
    lbfd_status st = set_device(c);
    if (st) return st;
    st = upload_field(c, c->L.phi, phi, c->N);
    if (st) return st;
    // solid flags for the sharp-interface mode (the threshold taken in FP64)
    c->solid.resize(c->N);
    for (size_t i = 0; i < c->N; ++i) c->solid[i] = phi[i] >= 0.5 ? 1 : 0;
    st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.solid), c->solid.data(), c->N,
                                     hipMemcpyHostToDevice, c->stream),
                   "upload solid flags");
    if (st) return st;
    st = hip_check(c, hipStreamSynchronize(c->stream), "upload solid flags");
    if (st) return st;
    c->mask_dirty = true;
    c->have_phi = true;
    return LBFD_OK;
}

lbfd_status lbfd_set_mechanism(lbfd_ctx* c, const lbfd_mechanism* m) {
    if (!c || !m) return LBFD_E_INVAL;
    if (m->n_species != c->ns) return fail(c, LBFD_E_INVAL, "mechanism species != grid species");
    HostMech h;
    std::string msg;
    lbfd_status st = mech_from_abi(m, h, msg);
    if (st) return fail(c, st, msg);
    if (c->have_params && (st = check_stable(c, c->params, &h))) return st;
    if ((st = set_device(c))) return st;
    HostMech old = c->mech;
    bool had = c->have_mech;
    c->mech = h;
    c->have_mech = true;
    st = upload_tables(c);
    if (st) {
        c->mech = old;
        c->have_mech = had;
        return st;
    }
    return LBFD_OK;
}

lbfd_status lbfd_set_params(lbfd_ctx* c, const lbfd_params* p) {
    if (!c || !p) return LBFD_E_INVAL;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(p->eta) || !pos(p->cp) || !pos(p->Pr) || !pos(p->rho_in) || !pos(p->T_in) ||
        !pos(p->nu_in) || !pos(p->T_solid) || !(p->sutherland_S >= 0.0))
        return fail(c, LBFD_E_INVAL, "eta, cp, Pr, rho_in, T_in, nu_in, T_solid must be positive");
    if (!(p->A_u >= 0.0) || !(p->A_T >= 0.0)) return fail(c, LBFD_E_INVAL, "negative coupling");
    if (p->mu_model != 0 && p->mu_model != 1) return fail(c, LBFD_E_INVAL, "mu_model");
    if (p->transport_model != 0 && p->transport_model != 1)
        return fail(c, LBFD_E_INVAL, "transport_model");
    if (p->n_sub < 1 || p->n_sub > 4096) return fail(c, LBFD_E_INVAL, "n_sub must be 1..4096");
    if (p->chem_scheme < 0 || p->chem_scheme > 2)
        return fail(c, LBFD_E_INVAL, "chem_scheme must be 0, 1 or 2");
    if (p->chem_scheme != 0 && c->nsm > 9)
        return fail(c, LBFD_E_UNSUPPORTED, "stiff reaction schemes: at most 9 species");
    const double tau_in = p->nu_in * 3.0 + 0.5;
    if (!(tau_in > 0.5 + 1e-3)) return fail(c, LBFD_E_INVAL, "relaxation time at the inlet <= 0.501");
    const double uin = std::sqrt(p->u_in[0] * p->u_in[0] + p->u_in[1] * p->u_in[1] +
                                 p->u_in[2] * p->u_in[2]);
    if (!(uin <= 0.1)) return fail(c, LBFD_E_INVAL, "|u_in| > 0.1 (low-Mach limit)");
    double im = 0.0;
    for (int k = 0; k < c->ns; ++k) {
        if (!pos(p->Le[k])) return fail(c, LBFD_E_INVAL, "Lewis numbers must be positive");
        if (!(p->Y_in[k] >= 0.0)) return fail(c, LBFD_E_INVAL, "negative inlet mass fraction");
        im += p->Y_in[k];
    }
    if (c->ns > 0 && !(std::fabs(im - 1.0) < 1e-6))
        return fail(c, LBFD_E_INVAL, "inlet mass fractions must sum to 1");
    for (int f = 0; f < 6; ++f)
        if (c->grid.fd_bc[f] == LBFD_FD_DIRICHLET && !pos(p->fd_face[f][0]))
            return fail(c, LBFD_E_INVAL, "Dirichlet face temperature must be positive");
    if (p->closed != 0 && p->closed != 1) return fail(c, LBFD_E_INVAL, "closed must be 0 or 1");
    if (p->closed) {
        for (int f = 0; f < 6; ++f)
            if (c->grid.lb_bc[f] == LBFD_LB_VELOCITY_INLET ||
                c->grid.lb_bc[f] == LBFD_LB_PRESSURE_OUTLET ||
                c->grid.lb_bc[f] == LBFD_LB_CHARACTERISTIC_OUTLET)
                return fail(c, LBFD_E_INVAL, "a closed domain has no inlet or outlet face");
        if (!(p->r_gas >= 0.0) || !(p->r_gas < p->cp))
            return fail(c, LBFD_E_INVAL, "closed domain: 0 <= r_gas < cp");
    }
    if (c->have_state && c->have_params && p->closed != c->params.closed)
        return fail(c, LBFD_E_STATE, "closing or opening the domain needs a new init_state");
    if (c->grid.lb_bc[1] == LBFD_LB_CHARACTERISTIC_OUTLET &&
        !(std::isfinite(p->outlet_sigma) && p->outlet_sigma > 0.0))
        return fail(c, LBFD_E_INVAL, "characteristic outlet: outlet_sigma must be > 0");
    if (!(p->T_max >= 0.0) || !std::isfinite(p->T_max))
        return fail(c, LBFD_E_INVAL, "T_max must be finite and >= 0");
    if (p->sharp_interface != 0 && p->sharp_interface != 1)
        return fail(c, LBFD_E_INVAL, "sharp_interface must be 0 or 1");
    if (p->sharp_interface && c->nsm > 4)
        return fail(c, LBFD_E_UNSUPPORTED, "sharp-interface mode: at most 4 species");
    if (p->sharp_interface)
        for (int f = 0; f < 6; ++f)
            if ((c->grid.lb_bc[f] == LBFD_LB_PERIODIC) != (c->grid.fd_bc[f] == LBFD_FD_PERIODIC))
                return fail(c, LBFD_E_UNSUPPORTED,
                            "sharp-interface mode: LB and FD must agree on periodic faces");
    if (p->sharp_interface && c->sur)
        return fail(c, LBFD_E_UNSUPPORTED,
                    "sharp-interface mode runs the exact reaction step (surrogate set)");
    lbfd_status st = check_stable(c, *p, c->have_mech ? &c->mech : nullptr);
    if (st) return st;
    st = set_device(c);
    if (st) return st;
    lbfd_params old = c->params;
    bool had = c->have_params;
    c->params = *p;
    c->have_params = true;
    if (p->sharp_interface != old.sharp_interface) c->mask_dirty = true;
    st = upload_tables(c);
    if (st) {
        c->params = old;
        c->have_params = had;
        return st;
    }
    return LBFD_OK;
}

lbfd_status lbfd_init_state(lbfd_ctx* c, const double* T, const double* Y, const double* u) {
    if (!c || !T) return LBFD_E_INVAL;
    if (c->ns > 0 && !Y) return fail(c, LBFD_E_INVAL, "Y required when n_species > 0");
    if (!c->have_phi || !ready_for_tables(c))
        return fail(c, LBFD_E_STATE, "phase field, params (and mechanism) must be set first");
    double tmin = INFINITY, tmax = 0.0;
    for (size_t i = 0; i < c->N; ++i) {
        if (!(T[i] > 0.0) || !std::isfinite(T[i]))
            return fail(c, LBFD_E_INVAL, "temperature must be positive and finite");
        tmin = std::min(tmin, T[i]);
        tmax = std::max(tmax, T[i]);
    }
    {  // the stability rule over the initial state's temperatures too
        lbfd_stability_report r;
        std::string msg;
        if (stability_eval(c->grid, c->params, c->have_mech ? &c->mech : nullptr, tmin, tmax, r,
                           msg))
            return fail(c, LBFD_E_INVAL, "initial state: " + msg);
    }
    lbfd_status st = set_device(c);
    if (st) return st;
    c->have_state = false;  // a failure below leaves no usable state
    // the temperature planes of this state hold T - T_ref (FP32 mode: the
    // solid temperature, fixed for the run; FP64 mode: 0)
    c->T_ref = c->fp32 ? c->params.T_solid : 0.0;
    if ((st = upload_tables(c))) return st;
    if ((st = upload_field(c, c->L.T0, T, c->N, c->T_ref))) return st;
    if (c->ns > 0 && (st = upload_field(c, c->L.Y0, Y, (size_t)c->ns * c->N))) return st;
    if (c->nsm > c->ns) {  // padded species planes of the kernel's bucket
        const size_t off = (size_t)c->ns * c->N * elem(c), len = (size_t)(c->nsm - c->ns) * c->N * elem(c);
        if ((st = hip_check(c, hipMemsetAsync(dptr<char>(c, c->L.Y0) + off, 0, len, c->stream), "clear")))
            return st;
        if ((st = hip_check(c, hipMemsetAsync(dptr<char>(c, c->L.Y1) + off, 0, len, c->stream), "clear")))
            return st;
    }
    if (u) {
        st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.scratch), u, c->dim * c->N * 8,
                                         hipMemcpyHostToDevice, c->stream),
                       "upload u");
        if (st) return st;
    }
    st = c->fp32 ? launch_init<float>(c, u != nullptr) : launch_init<double>(c, u != nullptr);
    if (st) return st;
    st = hip_check(c, hipMemsetAsync(dptr<char>(c, c->L.part), 0,
                                     (size_t)c->L.nslots * DIAG_STRIDE * sizeof(double), c->stream),
                   "clear diagnostics");
    if (st) return st;
    c->last_sur = false;
    st = hip_check(c, hipMemsetAsync(dptr<char>(c, c->L.count), 0, sizeof(int), c->stream),
                   "clear island count");
    if (st) return st;
    st = hip_check(c, hipMemsetAsync(dptr<char>(c, c->L.gtot), 0,
                                     (size_t)c->L.ngroups * GSPREAD * sizeof(int), c->stream),
                   "clear island group counts");
    if (st) return st;
    // characteristic outlet: the incoming wave amplitude starts at zero
    st = hip_check(c, hipMemsetAsync(dptr<char>(c, c->L.outw), 0,
                                     (size_t)c->grid.ny * c->grid.nz * sizeof(double), c->stream),
                   "clear outlet state");
    if (st) return st;
    st = hip_check(c, hipStreamSynchronize(c->stream), "init");
    if (st) return st;
    c->cur = 0;
    c->odd = 0;
    c->steps = 0;
    c->state_T[0] = tmin;
    c->state_T[1] = tmax;
    if (c->params.closed) {  // P0 = P0_in for the initial state; its sum of M / T
        const Par<double> pd = build_par<double>(c);
        P0State q{};
        q.p = q.p_prev = 1.0;
        q.rho_ref0 = pd.rho_ref;
        q.P0_in = pd.rho_ref * c->params.r_gas;
        st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.p0), &q, sizeof(q),
                                         hipMemcpyHostToDevice, c->stream),
                       "closed-domain state");
        if (st) return st;
        if ((st = launch_p0(c, 0))) return st;
        if ((st = hip_check(c, hipStreamSynchronize(c->stream), "closed-domain state"))) return st;
    }
    c->have_state = true;
    return LBFD_OK;
}

lbfd_status lbfd_get_p0_state(lbfd_ctx* c, double* out) {
    if (!c || !out) return LBFD_E_INVAL;
    if (!c->have_state || !c->params.closed)
        return fail(c, LBFD_E_STATE, "no closed-domain state");
    lbfd_status st = set_device(c);
    if (st) return st;
    P0State q;
    st = hip_check(c, hipMemcpyAsync(&q, dptr<char>(c, c->L.p0), sizeof(q), hipMemcpyDeviceToHost,
                                     c->stream),
                   "closed-domain state");
    if (st) return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "closed-domain state"))) return st;
    out[0] = q.S0;
    out[1] = q.p;
    out[2] = q.p_prev;
    return LBFD_OK;
}

lbfd_status lbfd_set_p0_state(lbfd_ctx* c, const double* in) {
    if (!c || !in) return LBFD_E_INVAL;
    if (!c->have_state || !c->params.closed)
        return fail(c, LBFD_E_STATE, "no closed-domain state");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(in[i]) || !(in[i] > 0.0))
            return fail(c, LBFD_E_INVAL, "closed-domain state must be positive");
    lbfd_status st = set_device(c);
    if (st) return st;
    P0State q;
    st = hip_check(c, hipMemcpyAsync(&q, dptr<char>(c, c->L.p0), sizeof(q), hipMemcpyDeviceToHost,
                                     c->stream),
                   "closed-domain state");
    if (st) return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "closed-domain state"))) return st;
    q.S0 = in[0];
    q.p = in[1];
    q.p_prev = in[2];
    st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.p0), &q, sizeof(q), hipMemcpyHostToDevice,
                                     c->stream),
                   "closed-domain state");
    if (st) return st;
    if ((st = launch_p0(c, 2))) return st;  // the parameter blocks follow the restored P0
    return hip_check(c, hipStreamSynchronize(c->stream), "closed-domain state");
}

lbfd_status lbfd_set_inlet_profile(lbfd_ctx* c, const double* u) {
    if (!c) return LBFD_E_INVAL;
    if (!u) {
        c->prof.clear();
        return LBFD_OK;
    }
    if (c->grid.lb_bc[0] != LBFD_LB_VELOCITY_INLET)
        return fail(c, LBFD_E_INVAL, "inlet profile without a velocity inlet on the -x face");
    if (c->nsm > 4) return fail(c, LBFD_E_UNSUPPORTED, "inlet profile: at most 4 species");
    if (c->have_mech && !c->mech.cp.empty())
        return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: no inlet profile");
    const size_t nr = (size_t)c->grid.ny * c->grid.nz;
    std::vector<double> prof(3 * nr, 0.0);
    for (size_t r = 0; r < nr; ++r) {
        double uu = 0.0;
        for (int a = 0; a < c->dim; ++a) {
            const double v = u[a * nr + r];
            if (!std::isfinite(v)) return fail(c, LBFD_E_INVAL, "non-finite inlet velocity");
            prof[a * nr + r] = v;
            uu += v * v;
        }
        if (!(std::sqrt(uu) <= 0.1))
            return fail(c, LBFD_E_INVAL, "inlet profile |u| > 0.1 (low-Mach limit)");
    }
    lbfd_status st = set_device(c);
    if (st) return st;
    std::vector<double> old;
    old.swap(c->prof);
    c->prof = prof;
    if ((st = upload_tables(c))) c->prof.swap(old);
    return st;
}

lbfd_status lbfd_set_outlet_wave(lbfd_ctx* c, const double* w) {
    if (!c || !w) return LBFD_E_INVAL;
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    if (c->grid.lb_bc[1] != LBFD_LB_CHARACTERISTIC_OUTLET)
        return fail(c, LBFD_E_INVAL, "no characteristic outlet");
    const size_t nr = (size_t)c->grid.ny * c->grid.nz;
    for (size_t i = 0; i < nr; ++i)
        if (!std::isfinite(w[i])) return fail(c, LBFD_E_INVAL, "non-finite outlet state");
    lbfd_status st = set_device(c);
    if (st) return st;
    st = hip_check(c, hipMemcpyAsync(dptr<char>(c, c->L.outw), w, nr * 8, hipMemcpyHostToDevice,
                                     c->stream),
                   "set outlet state");
    if (st) return st;
    return hip_check(c, hipStreamSynchronize(c->stream), "set outlet state");
}

lbfd_status lbfd_set_populations(lbfd_ctx* c, const double* g, const double* divu) {
    if (!c || !g) return LBFD_E_INVAL;
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    for (size_t i = 0; i < (size_t)c->Q * c->N; ++i)
        if (!std::isfinite(g[i])) return fail(c, LBFD_E_INVAL, "non-finite population");
    if (divu)
        for (size_t i = 0; i < c->N; ++i)
            if (!std::isfinite(divu[i])) return fail(c, LBFD_E_INVAL, "non-finite divergence");
    lbfd_status st = set_device(c);
    if (st) return st;
    if ((st = upload_field(c, c->L.g, g, (size_t)c->Q * c->N, 0.0, pop_scale(c)))) return st;
    if (divu && (st = upload_field(c, c->L.divu, divu, c->N))) return st;
    c->odd = 0;
    return LBFD_OK;
}

lbfd_status lbfd_step_phase(lbfd_ctx* c, int32_t n, int32_t phase) {
    if (!c || n < 0 || phase < 0 || phase > 7) return LBFD_E_INVAL;
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    lbfd_status st = set_device(c);
    if (st) return st;
    for (int i = 0; i < n; ++i) {
        st = c->fp32 ? launch_step<float>(c, phase) : launch_step<double>(c, phase);
        if (st) return st;
        c->cur ^= 1;
        if (phase & PH_LB) c->odd ^= 1;
        c->steps++;
        if (c->params.closed && (st = launch_p0(c, 1))) return st;  // P0 of the new state
    }
    return LBFD_OK;
}

lbfd_status lbfd_step(lbfd_ctx* c, int32_t n) { return lbfd_step_phase(c, n, LBFD_PHASE_ALL); }

lbfd_status lbfd_read(lbfd_ctx* c, int32_t field, int32_t comp, double* out) {
    if (!c || !out) return LBFD_E_INVAL;
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    lbfd_status st = set_device(c);
    if (st) return st;
    const size_t N = c->N, s = elem(c);
    switch (field) {
    case LBFD_F_T:
        return download_field(c, c->cur ? c->L.T1 : c->L.T0, out, N, c->T_ref);
    case LBFD_F_Y:
        if (comp < 0 || comp >= c->ns) return fail(c, LBFD_E_INVAL, "species index");
        return download_field(c, (c->cur ? c->L.Y1 : c->L.Y0) + comp * N * s, out, N);
    case LBFD_F_DIVU:
        return download_field(c, c->L.divu, out, N);
    case LBFD_F_OUTLET_WAVE: {
        const size_t nr = (size_t)c->grid.ny * c->grid.nz;
        st = hip_check(c, hipMemcpyAsync(out, dptr<double>(c, c->L.outw), nr * 8,
                                         hipMemcpyDeviceToHost, c->stream),
                       "read outlet state");
        if (st) return st;
        return hip_check(c, hipStreamSynchronize(c->stream), "read outlet state");
    }
    case LBFD_F_POPULATIONS: {
        if (comp < 0 || comp >= c->Q) return fail(c, LBFD_E_INVAL, "population index");
        // (the populations are stored scaled: 36 g in FP32 mode)
        if (!c->odd) return download_field(c, c->L.g + comp * N * s, out, N, 0.0, pop_scale(c));
        // swapped AA layout: natural g_i(x) sits in slot opp(i) of x - c_i, or
        // in the cell's own slot i when x - c_i is outside the domain
        std::vector<double> own(N), nb(N);
        const int i = comp, j = opp(comp);
        if ((st = download_field(c, c->L.g + i * N * s, own.data(), N, 0.0, pop_scale(c)))) return st;
        if ((st = download_field(c, c->L.g + j * N * s, nb.data(), N, 0.0, pop_scale(c)))) return st;
        const int* cx = c->dim == 2 ? Lat<2>::cx : Lat<3>::cx;
        const int* cy = c->dim == 2 ? Lat<2>::cy : Lat<3>::cy;
        const int* cz = c->dim == 2 ? Lat<2>::cz : Lat<3>::cz;
        const int n[3] = {c->grid.nx, c->grid.ny, c->grid.nz};
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x) {
                    int p[3] = {x - cx[i], y - cy[i], z - cz[i]};
                    bool inside = true;
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] >= 0 && p[a] < n[a]) continue;
                        if (c->grid.lb_bc[2 * a] == LBFD_LB_PERIODIC)
                            p[a] = (p[a] + n[a]) % n[a];
                        else
                            inside = false;
                    }
                    const size_t id = ((size_t)z * n[1] + y) * n[0] + x;
                    const size_t src = ((size_t)p[2] * n[1] + p[1]) * n[0] + p[0];
                    // sharp-interface mode: a solid cell keeps its own slots,
                    // a solid source is a wall
                    if (c->params.sharp_interface && inside)
                        inside = !c->solid[id] && !c->solid[src];
                    out[id] = inside ? nb[src] : own[id];
                }
        return LBFD_OK;
    }
    case LBFD_F_RHO:
    case LBFD_F_U:
    case LBFD_F_PH: {
        if (field == LBFD_F_U && (comp < 0 || comp >= c->dim))
            return fail(c, LBFD_E_INVAL, "velocity component");
        st = c->fp32 ? launch_macro<float>(c) : launch_macro<double>(c);
        if (st) return st;
        const int slot = field == LBFD_F_RHO ? 0 : field == LBFD_F_U ? 1 + comp : 4;
        st = hip_check(c, hipMemcpyAsync(out, dptr<double>(c, c->L.scratch) + slot * N, N * 8,
                                         hipMemcpyDeviceToHost, c->stream),
                       "read");
        if (st) return st;
        return hip_check(c, hipStreamSynchronize(c->stream), "read");
    }
    default:
        return fail(c, LBFD_E_INVAL, "unknown field");
    }
}

lbfd_status lbfd_diagnostics(lbfd_ctx* c, lbfd_diag* out) {
    if (!c || !out) return LBFD_E_INVAL;
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    lbfd_status st = set_device(c);
    if (st) return st;
    double* red = dptr<double>(c, c->L.red);
    const bool island = c->fp32 && c->ns > 0;
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(BLOCK), 0, c->stream,
                       dptr<double>(c, c->L.part), c->L.nblocks, island ? ISLAND_WG : 0,
                       island ? 2 * c->mlp_grid : 0, c->ns, red,
                       island ? dptr<int>(c, c->L.count) : (const int*)nullptr,
                       c->last_sur ? 1 : 0);
    if ((st = hip_check(c, hipGetLastError(), "diagnostics launch"))) return st;
    double h[DG_COUNT];
    st = hip_check(c, hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, c->stream),
                   "diagnostics");
    if (st) return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "diagnostics"))) return st;
    std::memset(out, 0, sizeof(*out));
    out->mass = h[DG_MASS];
    for (int k = 0; k < c->ns; ++k) out->species_mass[k] = h[DG_SP + k];
    out->enthalpy = h[DG_ENTH];
    out->kinetic = h[DG_KIN];
    out->umax = h[DG_UMAX];
    out->Tmin = h[DG_TMIN];
    out->Tmax = h[DG_TMAX];
    out->n_nonfinite = (int64_t)h[DG_NONFIN];
    out->n_tau_bad = (int64_t)h[DG_TAUBAD];
    out->n_negY = (int64_t)h[DG_NEGY];
    out->n_flagged_fp64 = (int64_t)h[DG_FLAG];
    out->n_fallback = (int64_t)h[DG_FALLBACK];
    for (int b = 0; b < 4; ++b) out->n_fallback_reason[b] = (int64_t)h[DG_FB_REASON + b];
    out->p0_ratio = 1.0;
    if (c->params.closed) {
        P0State q;
        st = hip_check(c, hipMemcpyAsync(&q, dptr<char>(c, c->L.p0), sizeof(q),
                                         hipMemcpyDeviceToHost, c->stream),
                       "closed-domain state");
        if (st) return st;
        if ((st = hip_check(c, hipStreamSynchronize(c->stream), "closed-domain state"))) return st;
        out->p0_ratio = q.p;
    }
    out->step = c->steps;
    if (out->n_nonfinite > 0) return fail(c, LBFD_E_NUMERIC, "non-finite values in the state");
    return LBFD_OK;
}

lbfd_status lbfd_synchronize(lbfd_ctx* c) {
    if (!c) return LBFD_E_INVAL;
    lbfd_status st = set_device(c);
    if (st) return st;
    return hip_check(c, hipStreamSynchronize(c->stream), "synchronize");
}

lbfd_status lbfd_step_bytes_per_cell(const lbfd_ctx* c, double* bytes) {
    if (!c || !bytes) return LBFD_E_INVAL;
    // populations read+write, T and Y read+write, divu read+write, phi read
    *bytes = (double)elem(c) * (2.0 * c->Q + 2.0 + 2.0 * c->nsm + 2.0 + 1.0);
    return LBFD_OK;
}

// ---------------------------------------------------------- surrogate
namespace {
uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__bf16 to_bf16(float f) {
    const uint16_t b = bf16_rne(f);
    __bf16 r;
    std::memcpy(&r, &b, 2);
    return r;
}
}  // namespace

lbfd_status lbfd_set_surrogate(lbfd_ctx* c, const float* w, const float* norm, const float* env) {
    if (!c) return LBFD_E_INVAL;
    if (!w) {
        c->sur = false;
        return LBFD_OK;
    }
    if (!norm || !env) return LBFD_E_INVAL;
    if (!c->fp32) return fail(c, LBFD_E_UNSUPPORTED, "the surrogate runs in FP32 mode only");
    if (c->have_params && c->params.sharp_interface)
        return fail(c, LBFD_E_UNSUPPORTED,
                    "sharp-interface mode runs the exact reaction step (no surrogate)");
    if (c->have_mech && !c->mech.cp.empty())
        return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: no surrogate");
    const int ns = c->ns, ni = 2 + ns, no = ns, H = MLP_H;
    if (ns < 1 || ni > MLP_KIN || no > MLP_OUT)
        return fail(c, LBFD_E_UNSUPPORTED, "surrogate needs 1..14 species");
    const float* W1 = w;
    const float* b1 = W1 + H * ni;
    const float* W2 = b1 + H;
    const float* b2 = W2 + H * H;
    const float* W3 = b2 + H;
    const float* b3 = W3 + no * H;
    const size_t nw = (size_t)(b3 + no - w);
    for (size_t i = 0; i < nw; ++i)
        if (!std::isfinite(w[i])) return fail(c, LBFD_E_INVAL, "non-finite surrogate weight");
    std::vector<SurWeights> hw(1);
    SurWeights& S = hw[0];
    std::memset(&S, 0, sizeof(S));
    for (int m = 0; m < MLP_HT; ++m)
        for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 8; ++j) {
                const int k = mlp_k1(l, j);
                S.w1[m][l][j] = to_bf16(k < ni ? W1[(32 * m + l % 32) * ni + k] : 0.f);
            }
    for (int m = 0; m < MLP_HT; ++m)
        for (int q = 0; q < MLP_HC; ++q)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j)
                    S.w2[m][q][l][j] =
                        to_bf16(W2[(32 * m + l % 32) * H + mlp_kh(q / 2, q % 2, l, j)]);
    for (int q = 0; q < MLP_HC; ++q)
        for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 8; ++j) {
                const int o = l % 32;
                S.w3[q][l][j] = to_bf16(o < no ? W3[o * H + mlp_kh(q / 2, q % 2, l, j)] : 0.f);
            }
    for (int i = 0; i < H; ++i) {
        S.b1[i] = b1[i];
        S.b2[i] = b2[i];
    }
    for (int o = 0; o < no; ++o) S.b3[o] = b3[o];
    SurPar P;
    std::memset(&P, 0, sizeof(P));
    P.n_in = ni;
    P.n_out = no;
    P.enabled = 1;
    for (int i = 0; i < ni; ++i) {
        const float sd = norm[ni + i];
        if (!(sd > 0.f) || !std::isfinite(norm[i]))
            return fail(c, LBFD_E_INVAL, "input standard deviation must be positive");
        P.mu_x[i] = norm[i];
        P.inv_sd_x[i] = 1.f / sd;
        // the training envelope, widened on both sides by 1 % of its range
        // plus 0.05 standard deviations of the input
        const float margin = 0.01f * (env[ni + i] - env[i]) + 0.05f * sd;
        if (!(margin >= 0.f)) return fail(c, LBFD_E_INVAL, "envelope with hi < lo");
        P.lo[i] = env[i] - margin;
        P.hi[i] = env[ni + i] + margin;
    }
    double sd_sum = 0.0;
    for (int o = 0; o < no; ++o) {
        P.mu_y[o] = norm[2 * ni + o];
        P.sd_y[o] = norm[2 * ni + no + o];
        if (!(P.sd_y[o] > 0.f) || !std::isfinite(P.mu_y[o]))
            return fail(c, LBFD_E_INVAL, "output standard deviation must be positive");
        sd_sum += P.sd_y[o];
    }
    P.p_in = 1.f;
    P.resid_tol = 0.05f;
    P.pos_tol = -1e-8f;
    P.sd_sum = (float)sd_sum;
    P.clip_tol = 0.05f;
    lbfd_status st = set_device(c);
    if (st) return st;
    if ((st = hip_check(c, hipMemcpyAsync(c->ws + c->L.sw, &S, sizeof(S), hipMemcpyHostToDevice,
                                          c->stream), "surrogate upload")))
        return st;
    if ((st = hip_check(c, hipMemcpyAsync(c->ws + c->L.sp, &P, sizeof(P), hipMemcpyHostToDevice,
                                          c->stream), "surrogate upload")))
        return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "surrogate upload"))) return st;
    c->sur = true;
    return LBFD_OK;
}

lbfd_status lbfd_surrogate_eval(lbfd_ctx* c, const float* T, const float* Y, int32_t n,
                                float* raw, float* omega, int32_t* fallback) {
    if (!c || n < 0 || (n > 0 && (!T || !Y || !raw || !omega || !fallback))) return LBFD_E_INVAL;
    if (!c->sur) return fail(c, LBFD_E_STATE, "no surrogate set");
    if (!c->have_params || (c->ns > 0 && !c->have_mech))
        return fail(c, LBFD_E_STATE, "params and mechanism first");
    if (n == 0) return LBFD_OK;
    lbfd_status st = set_device(c);
    if (st) return st;
    const int waves = (n + 63) / 64;
    const int grid = std::max(1, std::min(c->n_cu, (waves + 3) / 4));
    return hip_check(c, launch_mlp_eval_f32(c->nsm, T, Y, n, raw, omega, fallback,
                                            dptr<Par<float>>(c, c->L.parf),
                                            dptr<SurWeights>(c, c->L.sw), dptr<SurPar>(c, c->L.sp),
                                            grid, c->stream),
                     "surrogate eval launch");
}

lbfd_status lbfd_sample_states(lbfd_ctx* c, const int32_t* cells, int32_t n, float* x, float* y) {
    if (!c || n < 0 || (n > 0 && (!cells || !x || !y))) return LBFD_E_INVAL;
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    if (!c->fp32 || c->ns < 1 || 2 + c->ns > MLP_KIN || c->mech.nr < 1)
        return fail(c, LBFD_E_UNSUPPORTED, "sampling needs FP32 mode and a mechanism");
    if (!c->mech.cp.empty())
        return fail(c, LBFD_E_UNSUPPORTED, "species heat capacities: no surrogate sampling");
    if (n == 0) return LBFD_OK;
    lbfd_status st = set_device(c);
    if (st) return st;
    const float* T = dptr<float>(c, c->cur ? c->L.T1 : c->L.T0);
    const float* Y = dptr<float>(c, c->cur ? c->L.Y1 : c->L.Y0);
    return hip_check(c, launch_sample_f32(c->nsm, T, Y, (int)c->N, cells, n, x, y,
                                          dptr<Par<double>>(c, c->L.pard), 1.f, c->stream),
                     "sample launch");
}

// ---------------------------------------------------------- halo planes
// A slab of a decomposition along x holds one halo plane on each side (x = 0
// and x = nx - 1) around its own planes 1 .. nx - 2.  What a neighbour needs
// for the next step depends on the AA parity of the state:
//  - T and Y_k of the slab's own boundary plane, for the neighbour's halo;
//  - populations.  After an even (in-place) step the state is swapped: slot
//    opp(i) of a cell holds its post-collision g_i, and the next (odd) step
//    gathers the neighbour's from its halo cells: the own boundary plane's
//    slots with c_x = -face go to the same slots of the neighbour's halo
//    plane.  After an odd step the populations a slab pushed across the face
//    sit in its halo plane, slots with c_x = face; they belong in the same
//    slots of the neighbour's own boundary plane.
extern "C++" {
namespace {
template <typename R>
int halo_planes(lbfd_ctx* c, int face, bool pack, R** out, int* xs) {
    const size_t N = c->N;
    const int nx = c->grid.nx;
    const int own = face < 0 ? 1 : nx - 2, halo = face < 0 ? 0 : nx - 1;
    const bool swapped = c->odd != 0;  // the next step is odd
    // populations: which plane and which slots
    int pop_x, dir;
    if (swapped) {
        pop_x = pack ? own : halo;
        dir = pack ? -face : face;
    } else {
        pop_x = pack ? halo : own;
        dir = pack ? face : -face;
    }
    R* g = dptr<R>(c, c->L.g);
    const int* cx = c->dim == 2 ? Lat<2>::cx : Lat<3>::cx;
    int n = 0;
    for (int i = 0; i < c->Q; ++i)
        if (cx[i] == dir) {
            xs[n] = pop_x;
            out[n++] = g + (size_t)i * N;
        }
    const int tx = pack ? own : halo;
    xs[n] = tx;
    out[n++] = dptr<R>(c, c->cur ? c->L.T1 : c->L.T0);
    R* Y = dptr<R>(c, c->cur ? c->L.Y1 : c->L.Y0);
    for (int k = 0; k < c->ns; ++k) {
        xs[n] = tx;
        out[n++] = Y + (size_t)k * N;
    }
    return n;
}
template <typename R>
lbfd_status halo_copy(lbfd_ctx* c, int face, void* buf, int pack) {
    HaloArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.nplanes = halo_planes<R>(c, face, pack != 0, a.plane, a.xs);
    a.nx = c->grid.nx;
    a.ny = c->grid.ny;
    a.nz = c->grid.nz;
    a.buf = reinterpret_cast<R*>(buf);
    a.pack = pack;
    hipError_t e;
    if constexpr (sizeof(R) == 4)
        e = launch_halo_f32(a, c->stream);
    else
        e = launch_halo_f64(a, c->stream);
    return hip_check(c, e, "halo launch");
}
lbfd_status halo_entry(lbfd_ctx* c, int32_t face, const void* buf, int pack) {
    if (!c || !buf) return LBFD_E_INVAL;
    if (face != -1 && face != 1) return fail(c, LBFD_E_INVAL, "halo face must be -1 or +1");
    if (c->grid.nx < 3) return fail(c, LBFD_E_INVAL, "a slab needs nx >= 3 (two halo planes)");
    if (!c->have_state) return fail(c, LBFD_E_STATE, "init_state first");
    if (c->params.sharp_interface)
        return fail(c, LBFD_E_UNSUPPORTED,
                    "sharp-interface mode: the link masks do not cross slab faces");
    lbfd_status st = set_device(c);
    if (st) return st;
    void* b = const_cast<void*>(buf);
    return c->fp32 ? halo_copy<float>(c, face, b, pack) : halo_copy<double>(c, face, b, pack);
}
}  // namespace
}  // extern "C++"

lbfd_status lbfd_halo_bytes(const lbfd_ctx* c, size_t* bytes) {
    if (!c || !bytes) return LBFD_E_INVAL;
    const int nout = c->dim == 2 ? 3 : 5;
    *bytes = (size_t)(nout + 1 + c->ns) * c->grid.ny * c->grid.nz * elem(c);
    return LBFD_OK;
}

lbfd_status lbfd_halo_pack(lbfd_ctx* c, int32_t face, void* buf) {
    return halo_entry(c, face, buf, 1);
}

lbfd_status lbfd_halo_unpack(lbfd_ctx* c, int32_t face, const void* buf) {
    return halo_entry(c, face, buf, 0);
}

lbfd_status lbfd_set_timing(lbfd_ctx* c, int32_t enable) {
    if (!c) return LBFD_E_INVAL;
    c->timing = enable != 0;
    c->ev_used[0] = c->ev_used[1] = c->ev_used[2] = 0;
    return LBFD_OK;
}

lbfd_status lbfd_kernel_time(lbfd_ctx* c, int32_t kernel, int64_t* launches, double* mean_ms) {
    if (!c || !launches || !mean_ms || kernel < 0 || kernel > 2) return LBFD_E_INVAL;
    lbfd_status st = set_device(c);
    if (st) return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "kernel time"))) return st;
    double sum = 0.0;
    const size_t n = c->ev_used[kernel];
    for (size_t i = 0; i < n; ++i) {
        float ms = 0.f;
        st = hip_check(c, hipEventElapsedTime(&ms, c->ev[kernel][2 * i], c->ev[kernel][2 * i + 1]),
                       "kernel time");
        if (st) return st;
        sum += ms;
    }
    *launches = (int64_t)n;
    *mean_ms = n ? sum / (double)n : 0.0;
    return LBFD_OK;
}

lbfd_status lbfd_destroy(lbfd_ctx* c) {
    if (c) {
        if (set_device(c) == LBFD_OK)
            for (auto& v : c->ev)
                for (hipEvent_t e : v) (void)hipEventDestroy(e);
    }
    delete c;
    return LBFD_OK;
}

const char* lbfd_last_error(const lbfd_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
