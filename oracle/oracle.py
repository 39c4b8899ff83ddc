"""ctypes wrapper of the FP64 CPU oracle (liblbfd_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It marshals a setup
dictionary (as produced by the seeded input generators) into the oracle's own
C struct; it shares no code with the HIP binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbfd_oracle.so")
SRC = os.path.join(HERE, "lbfd_oracle.c")

MAXS, MAXR = 16, 32
LB = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3, "char_outlet": 4}
FD = {"periodic": 0, "dirichlet": 1, "neumann": 2}
PH_LB, PH_FD, PH_CHEM, PH_ALL = 1, 2, 4, 7
F_RHO, F_U, F_T, F_Y, F_PH, F_POP, F_DIVU, F_OUTW = range(8)
D_MASS, D_SPECIES, D_ENTHALPY, D_KINETIC, D_UMAX, D_TMIN, D_TMAX = 0, 1, 17, 18, 19, 20, 21
D_NONFINITE, D_TAUBAD, D_NEGY, D_FLAGGED, D_FALLBACK, D_STEP, D_LEN = 22, 23, 24, 25, 26, 27, 28


class Setup(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ns", C.c_int32), ("nr", C.c_int32),
        ("lb_bc", C.c_int32 * 6), ("fd_bc", C.c_int32 * 6),
        ("fd_val", (C.c_double * (1 + MAXS)) * 6),
        ("A_u", C.c_double), ("A_T", C.c_double), ("eta", C.c_double), ("T_s", C.c_double),
        ("Pr", C.c_double), ("cp", C.c_double), ("rho_in", C.c_double), ("T_in", C.c_double),
        ("nu_in", C.c_double), ("S_suth", C.c_double),
        ("mu_model", C.c_int32), ("transport", C.c_int32),
        ("u_in", C.c_double * 3), ("F_b", C.c_double * 3),
        ("Y_in", C.c_double * MAXS), ("Le", C.c_double * MAXS),
        ("n_sub", C.c_int32), ("theta_ign", C.c_double),
        ("M", C.c_double * MAXS), ("dhf", C.c_double * MAXS), ("mu_star", C.c_double * MAXS),
        ("nu_f", (C.c_int32 * MAXS) * MAXR), ("nu_r", (C.c_int32 * MAXS) * MAXR),
        ("A", C.c_double * MAXR), ("beta", C.c_double * MAXR), ("theta", C.c_double * MAXR),
        ("rev", C.c_int32 * MAXR), ("lnKc_a", C.c_double * MAXR), ("lnKc_b", C.c_double * MAXR),
        ("closed", C.c_int32), ("r_gas", C.c_double), ("p0", C.c_double),
        ("si", C.c_int32), ("outlet_sigma", C.c_double), ("chem_scheme", C.c_int32),
        ("cpk", C.c_int32), ("cp_k", C.c_double * MAXS),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", LIB_PATH, SRC, "-lm"]
        subprocess.check_call(cmd)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Setup), dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_set_populations.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_inlet_profile.argtypes = [C.c_void_p, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.orc_read.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp]
        L.orc_diag.argtypes = [C.c_void_p, dp]
        L.orc_nthreads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_eq_source.argtypes = [C.c_int32, C.c_double, dp, C.c_double, dp, dp, C.c_double,
                                    dp, dp]
        L.orc_lattice.argtypes = [C.c_int32, C.POINTER(C.c_int32), dp]
        L.orc_mixture.argtypes = [C.POINTER(Setup), C.c_double, dp, dp, dp, dp]
        L.orc_eos.restype = C.c_double
        L.orc_eos.argtypes = [C.POINTER(Setup), C.c_double, dp]
        L.orc_reactor.argtypes = [C.POINTER(Setup), dp, dp, C.c_int32]
        L.orc_rates.argtypes = [C.POINTER(Setup), C.c_double, dp, C.c_double, dp, dp]
        L.orc_rates_jacobian.argtypes = [C.POINTER(Setup), C.c_double, dp, C.c_double, dp, dp]
        L.orc_fd_only.argtypes = [C.c_void_p, dp, dp]
        L.orc_p0.restype = C.c_double
        L.orc_p0.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_setup(s: dict) -> Setup:
    st = Setup()
    st.dim, st.nx, st.ny, st.nz = s["dim"], s["nx"], s["ny"], s["nz"]
    ns = st.ns = s["ns"]
    mech = s["mech"]
    nr = st.nr = len(mech["A"])
    for f in range(6):
        st.lb_bc[f] = LB[s["lb_bc"][f]]
        st.fd_bc[f] = FD[s["fd_bc"][f]]
        for j, v in enumerate(s["fd_val"][f]):
            st.fd_val[f][j] = v
    for k in ("A_u", "A_T", "eta", "T_s", "Pr", "cp", "rho_in", "T_in", "nu_in", "S_suth",
              "theta_ign"):
        setattr(st, k, float(s[k]))
    st.mu_model, st.transport, st.n_sub = s["mu_model"], s["transport"], s["n_sub"]
    for a in range(3):
        st.u_in[a] = s["u_in"][a]
        st.F_b[a] = s["F_b"][a]
    for k in range(ns):
        st.Y_in[k] = s["Y_in"][k]
        st.Le[k] = s["Le"][k]
        st.M[k] = mech["M"][k]
        st.dhf[k] = mech["dhf"][k]
        st.mu_star[k] = mech["mu_star"][k]
    for j in range(nr):
        for k in range(ns):
            st.nu_f[j][k] = mech["nu_f"][j][k]
            st.nu_r[j][k] = mech["nu_r"][j][k]
        st.A[j], st.beta[j], st.theta[j] = mech["A"][j], mech["beta"][j], mech["theta"][j]
        st.rev[j] = mech["rev"][j]
        st.lnKc_a[j], st.lnKc_b[j] = mech["lnKc_a"][j], mech["lnKc_b"][j]
    st.closed = int(s.get("closed", 0))
    st.r_gas = float(s.get("r_gas", 0.0))
    st.p0 = 1.0
    st.si = int(s.get("si", 0))
    st.outlet_sigma = float(s.get("outlet_sigma", 0.0))
    st.chem_scheme = int(s.get("chem_scheme", 0))
    cpk = mech.get("cp")
    st.cpk = 1 if cpk is not None else 0
    if cpk is not None:
        for k in range(ns):
            st.cp_k[k] = float(cpk[k])
    return st


class Oracle:
    """One oracle simulation context (FP64, two-array pull streaming)."""

    def __init__(self, setup: dict, phi: np.ndarray):
        self.setup = setup
        self._st = make_setup(setup)
        self.dim, self.ns = setup["dim"], setup["ns"]
        self.Q = 9 if self.dim == 2 else 19
        self.shape = (setup["nz"], setup["ny"], setup["nx"])
        self.N = int(np.prod(self.shape))
        ph = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.N)
        self._h = lib().orc_create(C.byref(self._st), _dp(ph))
        if not self._h:
            raise ValueError("oracle rejected the setup")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def init_state(self, T, Y=None, u=None):
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.N)
        Yb = np.ascontiguousarray(Y if Y is not None and self.ns else np.zeros(1),
                                  dtype=np.float64).reshape(-1)
        ub = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        lib().orc_init_state(self._h, _dp(T), _dp(Yb), None if ub is None else _dp(ub))

    def set_populations(self, g, divu=None):
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        assert g.size == self.Q * self.N
        d = None if divu is None else np.ascontiguousarray(divu, dtype=np.float64).reshape(-1)
        lib().orc_set_populations(self._h, _dp(g), None if d is None else _dp(d))

    def set_inlet_profile(self, u):
        """Velocity of each inlet row, u[a][z][y] for a < dim (None: uniform u_in)."""
        if u is None:
            lib().orc_set_inlet_profile(self._h, None)
            return
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        assert u.size == self.dim * self.shape[0] * self.shape[1]
        self._uprof = u
        lib().orc_set_inlet_profile(self._h, _dp(u))

    def step(self, n=1, mask=PH_ALL):
        lib().orc_step(self._h, int(n), int(mask))

    def read(self, field, comp=0):
        out = np.empty(self.N, np.float64)
        if lib().orc_read(self._h, field, comp, _dp(out)) != 0:
            raise ValueError("bad field/component")
        return out.reshape(self.shape)

    def fields(self):
        d = {"rho": self.read(F_RHO), "T": self.read(F_T), "Ph": self.read(F_PH),
             "divu": self.read(F_DIVU)}
        d["u"] = np.stack([self.read(F_U, a) for a in range(self.dim)])
        if self.ns:
            d["Y"] = np.stack([self.read(F_Y, k) for k in range(self.ns)])
        return d

    def outlet_wave(self):
        """Characteristic outlet: incoming wave amplitude per outlet row [nz][ny]."""
        out = np.empty(self.N, np.float64)
        lib().orc_read(self._h, F_OUTW, 0, _dp(out))
        return out[: self.shape[0] * self.shape[1]].reshape(self.shape[:2]).copy()

    def populations(self):
        return np.stack([self.read(F_POP, i) for i in range(self.Q)])

    def diag(self):
        out = np.empty(D_LEN, np.float64)
        lib().orc_diag(self._h, _dp(out))
        return out

    def p0(self):
        """P0 / P0_in of the current state (1 unless the domain is closed)."""
        return float(lib().orc_p0(self._h))

    def fd_only(self):
        Ts = np.empty(self.N)
        Ys = np.empty(max(self.ns, 1) * self.N)
        lib().orc_fd_only(self._h, _dp(Ts), _dp(Ys))
        return Ts.reshape(self.shape), Ys[: self.ns * self.N].reshape((self.ns,) + self.shape)


def eq_source(dim, rho, u, Ph, G, F, divu):
    Q = 9 if dim == 2 else 19
    geq, xi = np.empty(Q), np.empty(Q)
    arr = lambda v: np.ascontiguousarray(np.resize(np.asarray(v, float), 3))
    lib().orc_eq_source(dim, rho, _dp(arr(u)), Ph, _dp(arr(G)), _dp(arr(F)), divu, _dp(geq),
                        _dp(xi))
    return geq, xi


def lattice(dim):
    Q = 9 if dim == 2 else 19
    c = np.empty(3 * Q, np.int32)
    w = np.empty(Q)
    lib().orc_lattice(dim, c.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return c.reshape(Q, 3), w


def mixture(setup, T, Y):
    st = make_setup(setup)
    ns = setup["ns"]
    Yb = np.ascontiguousarray(np.asarray(Y, float) if ns else np.zeros(1))
    mu, lam = np.zeros(1), np.zeros(1)
    rD = np.zeros(max(ns, 1))
    lib().orc_mixture(C.byref(st), float(T), _dp(Yb), _dp(mu), _dp(lam), _dp(rD))
    return float(mu[0]), float(lam[0]), rD[:ns]


def eos(setup, T, Y):
    st = make_setup(setup)
    Yb = np.ascontiguousarray(np.asarray(Y, float) if setup["ns"] else np.zeros(1))
    return lib().orc_eos(C.byref(st), float(T), _dp(Yb))


def rates(setup, T, Y, rho):
    """Production rates omega_k and heat release omega_T (Eqs. 8 and 9)."""
    st = make_setup(setup)
    Yb = np.ascontiguousarray(np.asarray(Y, float))
    wk = np.zeros(max(setup["ns"], 1))
    wT = np.zeros(1)
    lib().orc_rates(C.byref(st), float(T), _dp(Yb), float(rho), _dp(wk), _dp(wT))
    return wk[: setup["ns"]], float(wT[0])


def rates_jacobian(setup, T, Y, rho):
    """f = (omega_k/rho, omega_T/(rho cp)) and J = df/dy, y = (Y, T), at fixed rho."""
    st = make_setup(setup)
    n = setup["ns"] + 1
    Yb = np.ascontiguousarray(np.asarray(Y, float))
    f = np.zeros(n)
    J = np.zeros(n * n)
    lib().orc_rates_jacobian(C.byref(st), float(T), _dp(Yb), float(rho), _dp(f), _dp(J))
    return f, J.reshape(n, n)


def reactor(setup, T, Y, nsteps):
    """0-D isobaric reactor: nsteps steps of the reaction step (its scheme)."""
    st = make_setup(setup)
    Tb = np.array([float(T)])
    Yb = np.ascontiguousarray(np.asarray(Y, float).copy())
    lib().orc_reactor(C.byref(st), _dp(Tb), _dp(Yb), int(nsteps))
    return float(Tb[0]), Yb


def nthreads():
    return int(lib().orc_nthreads())


def set_threads(n):
    """OpenMP threads of the oracle's next steps."""
    lib().orc_set_threads(int(n))
