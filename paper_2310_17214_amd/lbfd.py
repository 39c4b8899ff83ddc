"""Python binding of the C ABI in include/lbfd.h (liblbfd_hip.so).

Argument marshalling only: every step of the coupled update runs in the HIP
kernels of the library.  PyTorch provides the device workspace (a uint8 CUDA
tensor) and the stream.  The library is loaded from the package directory;
if it has not been built, importing this module fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbfd_hip.so")
MAX_SPECIES, MAX_REACTIONS = 16, 32

LBFD_OK, LBFD_E_INVAL, LBFD_E_NOMEM, LBFD_E_DEVICE = 0, -1, -2, -3
LBFD_E_STATE, LBFD_E_NUMERIC, LBFD_E_UNSUPPORTED = -4, -5, -6
STATUS = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_STATE",
          -5: "E_NUMERIC", -6: "E_UNSUPPORTED"}
FP64, FP32 = 0, 1
F_RHO, F_U, F_T, F_Y, F_PH, F_POPULATIONS, F_DIVU, F_OUTLET_WAVE = range(8)
PHASE_LB, PHASE_FD, PHASE_CHEM, PHASE_ALL = 1, 2, 4, 7
LB_BC = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3, "char_outlet": 4}
FD_BC = {"periodic": 0, "dirichlet": 1, "neumann": 2}

EXPORTED = ["lbfd_workspace_bytes", "lbfd_create", "lbfd_set_phase_field", "lbfd_set_mechanism",
            "lbfd_set_params", "lbfd_init_state", "lbfd_set_populations", "lbfd_set_inlet_profile",
            "lbfd_set_outlet_wave",
            "lbfd_get_p0_state", "lbfd_set_p0_state", "lbfd_step",
            "lbfd_step_phase", "lbfd_read", "lbfd_diagnostics", "lbfd_synchronize",
            "lbfd_step_bytes_per_cell", "lbfd_set_timing", "lbfd_kernel_time",
            "lbfd_set_surrogate", "lbfd_surrogate_eval", "lbfd_sample_states",
            "lbfd_halo_bytes", "lbfd_halo_pack", "lbfd_halo_unpack",
            "lbfd_trainer_workspace_bytes", "lbfd_trainer_create", "lbfd_trainer_fit_norm",
            "lbfd_trainer_set_weights", "lbfd_trainer_step", "lbfd_trainer_gradient",
            "lbfd_trainer_export", "lbfd_trainer_destroy", "lbfd_trainer_last_error",
            "lbfd_destroy", "lbfd_last_error", "lbfd_stability", "lbfd_fit_norm_noalloc"]
LBFD_KERNEL_STEP, LBFD_KERNEL_ISLAND, LBFD_KERNEL_SURROGATE = 0, 1, 2


class TrainCfg(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("batch", C.c_int32), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("precision", C.c_int32), ("n_species", C.c_int32),
                ("lb_bc", C.c_int32 * 6), ("fd_bc", C.c_int32 * 6)]


class Params(C.Structure):
    _fields_ = [("A_u", C.c_double), ("A_T", C.c_double), ("eta", C.c_double),
                ("T_solid", C.c_double), ("Pr", C.c_double), ("cp", C.c_double),
                ("rho_in", C.c_double), ("T_in", C.c_double), ("nu_in", C.c_double),
                ("sutherland_S", C.c_double), ("mu_model", C.c_int32),
                ("transport_model", C.c_int32), ("u_in", C.c_double * 3),
                ("body_force", C.c_double * 3), ("Y_in", C.c_double * MAX_SPECIES),
                ("Le", C.c_double * MAX_SPECIES),
                ("fd_face", (C.c_double * (1 + MAX_SPECIES)) * 6),
                ("n_sub", C.c_int32), ("ign_threshold", C.c_double),
                ("closed", C.c_int32), ("r_gas", C.c_double), ("T_max", C.c_double),
                ("chem_scheme", C.c_int32), ("outlet_sigma", C.c_double),
                ("sharp_interface", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class StabilityReport(C.Structure):
    _fields_ = [("T_lo", C.c_double), ("T_hi", C.c_double), ("tau_lo", C.c_double),
                ("alpha_hi", C.c_double), ("D_hi", C.c_double), ("h_hi", C.c_double),
                ("u_sum", C.c_double), ("fd_sum", C.c_double), ("kappa_hi", C.c_double),
                ("h_kappa", C.c_double), ("violated", C.c_int32)]


class Mechanism(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("M", _dp), ("dhf", _dp), ("mu_star", _dp), ("nu_f", _ip), ("nu_r", _ip),
                ("A", _dp), ("beta", _dp), ("theta", _dp), ("reversible", _ip),
                ("lnKc_a", _dp), ("lnKc_b", _dp), ("cp", _dp)]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("species_mass", C.c_double * MAX_SPECIES),
                ("enthalpy", C.c_double), ("kinetic", C.c_double), ("umax", C.c_double),
                ("Tmin", C.c_double), ("Tmax", C.c_double), ("n_nonfinite", C.c_int64),
                ("n_tau_bad", C.c_int64), ("n_negY", C.c_int64), ("n_flagged_fp64", C.c_int64),
                ("n_fallback", C.c_int64), ("step", C.c_int64),
                ("n_fallback_reason", C.c_int64 * 4), ("p0_ratio", C.c_double)]


_lib = None


def lib():
    """Load liblbfd_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int
        L.lbfd_workspace_bytes.argtypes = [C.POINTER(Grid), C.POINTER(C.c_size_t)]
        L.lbfd_create.argtypes = [C.POINTER(Grid), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbfd_set_phase_field.argtypes = [vp, _dp]
        L.lbfd_set_mechanism.argtypes = [vp, C.POINTER(Mechanism)]
        L.lbfd_set_params.argtypes = [vp, C.POINTER(Params)]
        L.lbfd_init_state.argtypes = [vp, _dp, _dp, _dp]
        L.lbfd_set_populations.argtypes = [vp, _dp, _dp]
        L.lbfd_set_inlet_profile.argtypes = [vp, _dp]
        L.lbfd_set_outlet_wave.argtypes = [vp, _dp]
        L.lbfd_get_p0_state.argtypes = [vp, _dp]
        L.lbfd_set_p0_state.argtypes = [vp, _dp]
        L.lbfd_step.argtypes = [vp, C.c_int32]
        L.lbfd_step_phase.argtypes = [vp, C.c_int32, C.c_int32]
        L.lbfd_read.argtypes = [vp, C.c_int32, C.c_int32, _dp]
        L.lbfd_diagnostics.argtypes = [vp, C.POINTER(Diag)]
        L.lbfd_synchronize.argtypes = [vp]
        L.lbfd_step_bytes_per_cell.argtypes = [vp, _dp]
        _fp = C.POINTER(C.c_float)
        L.lbfd_set_surrogate.argtypes = [vp, _fp, _fp, _fp]
        L.lbfd_surrogate_eval.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp]
        L.lbfd_sample_states.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.lbfd_halo_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.lbfd_halo_pack.argtypes = [vp, C.c_int32, vp]
        L.lbfd_halo_unpack.argtypes = [vp, C.c_int32, vp]
        L.lbfd_trainer_workspace_bytes.argtypes = [C.POINTER(TrainCfg), C.POINTER(C.c_size_t)]
        L.lbfd_trainer_create.argtypes = [C.POINTER(TrainCfg), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbfd_trainer_fit_norm.argtypes = [vp, vp, vp, C.c_int32]
        L.lbfd_trainer_set_weights.argtypes = [vp, _fp]
        L.lbfd_trainer_step.argtypes = [vp, vp, vp, C.c_int32, vp, C.c_float, _dp]
        L.lbfd_trainer_gradient.argtypes = [vp, vp, vp, C.c_int32, vp, _fp, _dp]
        L.lbfd_trainer_export.argtypes = [vp, _fp, _fp, _fp]
        L.lbfd_trainer_destroy.argtypes = [vp]
        L.lbfd_trainer_last_error.argtypes = [vp]
        L.lbfd_trainer_last_error.restype = C.c_char_p
        L.lbfd_set_timing.argtypes = [vp, C.c_int32]
        L.lbfd_kernel_time.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), _dp]
        L.lbfd_stability.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.POINTER(Mechanism),
                                     C.c_double, C.c_double, C.POINTER(StabilityReport)]
        L.lbfd_fit_norm_noalloc.argtypes = [C.c_int32, vp, vp, C.c_int32, _fp, _fp, vp]
        L.lbfd_destroy.argtypes = [vp]
        L.lbfd_last_error.argtypes = [vp]
        L.lbfd_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name != "lbfd_last_error":
                getattr(L, name).restype = st
        _lib = L
    return _lib


class LbfdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def make_grid(s: dict) -> Grid:
    g = Grid()
    g.dim, g.nx, g.ny, g.nz = s["dim"], s["nx"], s["ny"], s["nz"]
    g.precision = FP32 if s.get("precision", "fp64") == "fp32" else FP64
    g.n_species = s["ns"]
    for f in range(6):
        g.lb_bc[f] = LB_BC[s["lb_bc"][f]]
        g.fd_bc[f] = FD_BC[s["fd_bc"][f]]
    return g


def make_params(s: dict) -> Params:
    p = Params()
    p.A_u, p.A_T, p.eta, p.T_solid = s["A_u"], s["A_T"], s["eta"], s["T_s"]
    p.Pr, p.cp, p.rho_in, p.T_in = s["Pr"], s["cp"], s["rho_in"], s["T_in"]
    p.nu_in, p.sutherland_S = s["nu_in"], s["S_suth"]
    p.mu_model, p.transport_model = s["mu_model"], s["transport"]
    for a in range(3):
        p.u_in[a] = s["u_in"][a]
        p.body_force[a] = s["F_b"][a]
    for k in range(s["ns"]):
        p.Y_in[k] = s["Y_in"][k]
        p.Le[k] = s["Le"][k]
    for f in range(6):
        for j, v in enumerate(s["fd_val"][f]):
            p.fd_face[f][j] = v
    p.n_sub, p.ign_threshold = s["n_sub"], s["theta_ign"]
    p.closed, p.r_gas = int(s.get("closed", 0)), float(s.get("r_gas", 0.0))
    p.T_max = float(s.get("T_max", 0.0))
    p.sharp_interface = int(s.get("si", 0))
    p.outlet_sigma = float(s.get("outlet_sigma", 0.0))
    p.chem_scheme = int(s.get("chem_scheme", 0))
    return p


class _MechArrays:
    """Keeps the numpy tables alive while the struct points at them."""

    def __init__(self, s: dict):
        m, ns = s["mech"], s["ns"]
        nr = len(m["A"])
        f64 = lambda v, n: np.ascontiguousarray(np.resize(np.asarray(v, np.float64), max(n, 1)))
        i32 = lambda v, n: np.ascontiguousarray(np.resize(np.asarray(v, np.int32).reshape(-1),
                                                          max(n, 1)))
        self.arrs = dict(M=f64(m["M"], ns), dhf=f64(m["dhf"], ns), mu_star=f64(m["mu_star"], ns),
                         nu_f=i32(m["nu_f"] if nr else [0], nr * ns),
                         nu_r=i32(m["nu_r"] if nr else [0], nr * ns),
                         A=f64(m["A"] if nr else [0], nr), beta=f64(m["beta"] if nr else [0], nr),
                         theta=f64(m["theta"] if nr else [0], nr),
                         reversible=i32(m["rev"] if nr else [0], nr),
                         lnKc_a=f64(m["lnKc_a"] if nr else [0], nr),
                         lnKc_b=f64(m["lnKc_b"] if nr else [0], nr))
        if m.get("cp") is not None:
            self.arrs["cp"] = f64(m["cp"], ns)
        st = Mechanism()
        st.n_species, st.n_reactions = ns, nr
        for k, a in self.arrs.items():
            setattr(st, k, a.ctypes.data_as(_ip if a.dtype == np.int32 else _dp))
        self.struct = st


def fit_norm_noalloc(n_species, x, y, stream=None):
    """Normalisation statistics and envelope of training pairs (torch float32
    CUDA tensors x [n, 2 + ns], y [n, ns]) through the entry point that
    allocates nothing: (norm, envelope) as numpy float32 arrays."""
    import torch

    ni = 2 + n_species
    x, y = x.contiguous(), y.contiguous()
    nrm = np.empty(2 * ni + 2 * n_species, np.float32)
    env = np.empty(2 * ni, np.float32)
    s = stream if stream is not None else torch.cuda.current_stream()
    fp = C.POINTER(C.c_float)
    st = lib().lbfd_fit_norm_noalloc(int(n_species), x.data_ptr(), y.data_ptr(), int(x.shape[0]),
                                     nrm.ctypes.data_as(fp), env.ctypes.data_as(fp),
                                     C.c_void_p(s.cuda_stream))
    if st != LBFD_OK:
        raise LbfdError(st, "fit_norm_noalloc")
    return nrm, env


def stability(setup: dict, T_lo=0.0, T_hi=0.0):
    """The library's explicit-stability rule for a setup (host only, no
    device): (status, report dict) with status LBFD_OK or LBFD_E_INVAL."""
    g = make_grid(setup)
    p = make_params(setup)
    m = _MechArrays(setup) if setup["ns"] > 0 else None
    r = StabilityReport()
    st = lib().lbfd_stability(C.byref(g), C.byref(p), C.byref(m.struct) if m else None,
                              float(T_lo), float(T_hi), C.byref(r))
    return st, {k: getattr(r, k) for k, _ in StabilityReport._fields_}


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


class Context:
    """One simulation on one GPU: owns a torch workspace and a C context."""

    def __init__(self, setup: dict, phi: np.ndarray, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        L = lib()
        self.setup = setup
        self.dim, self.ns = setup["dim"], setup["ns"]
        self.Q = 9 if self.dim == 2 else 19
        self.shape = (setup["nz"], setup["ny"], setup["nx"])
        self.N = int(np.prod(self.shape))
        self.precision = "fp32" if setup.get("precision", "fp64") == "fp32" else "fp64"
        self._grid = make_grid(setup)
        nbytes = C.c_size_t()
        self._check(L.lbfd_workspace_bytes(C.byref(self._grid), C.byref(nbytes)), None)
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self._ptr = base + (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        self._check(L.lbfd_create(C.byref(self._grid), C.c_void_p(self._ptr), nbytes.value,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self._h = h
        self._lib = L
        self._check(L.lbfd_set_phase_field(h, _f64(phi).ctypes.data_as(_dp)))
        if self.ns > 0:
            self._mech = _MechArrays(setup)
            self._check(L.lbfd_set_mechanism(h, C.byref(self._mech.struct)))
        self._params = make_params(setup)
        self._check(L.lbfd_set_params(h, C.byref(self._params)))

    def set_params(self, setup):
        """Re-upload the physical and coupling parameters (same grid and
        mechanism), e.g. a new ignition threshold between steps."""
        self._params = make_params(setup)
        self._check(lib().lbfd_set_params(self._h, C.byref(self._params)))

    def _check(self, status, h="self"):
        if status != LBFD_OK:
            handle = self._h if h == "self" else None
            msg = lib().lbfd_last_error(handle).decode() if handle else ""
            raise LbfdError(status, msg)

    def __del__(self):
        # the library handle is kept on the object: module globals may already
        # be gone when this runs at interpreter exit
        h, L = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h and L is not None:
            try:
                L.lbfd_synchronize(h)
            finally:
                L.lbfd_destroy(h)
            self._h = None

    def init_state(self, T, Y=None, u=None):
        T = _f64(T)
        Yb = _f64(Y) if (Y is not None and self.ns) else None
        ub = _f64(u) if u is not None else None
        self._check(lib().lbfd_init_state(self._h, T.ctypes.data_as(_dp),
                                          None if Yb is None else Yb.ctypes.data_as(_dp),
                                          None if ub is None else ub.ctypes.data_as(_dp)))

    def set_populations(self, g, divu=None):
        g = _f64(g)
        d = _f64(divu) if divu is not None else None
        self._check(lib().lbfd_set_populations(self._h, g.ctypes.data_as(_dp),
                                               None if d is None else d.ctypes.data_as(_dp)))

    def set_inlet_profile(self, u):
        """Velocity of each inlet row, u[a][z][y] for a < dim (None: uniform u_in)."""
        if u is None:
            self._check(lib().lbfd_set_inlet_profile(self._h, None))
            return
        u = _f64(u)
        self._check(lib().lbfd_set_inlet_profile(self._h, u.ctypes.data_as(_dp)))

    def p0_state(self):
        """Closed domain: (S0, p, p_prev) for a checkpoint."""
        out = np.zeros(3)
        self._check(lib().lbfd_get_p0_state(self._h, out.ctypes.data_as(_dp)))
        return out

    def set_p0_state(self, st):
        st = _f64(st)
        self._check(lib().lbfd_set_p0_state(self._h, st.ctypes.data_as(_dp)))

    def step(self, n=1):
        self._check(lib().lbfd_step(self._h, int(n)))

    def step_phase(self, n, mask):
        self._check(lib().lbfd_step_phase(self._h, int(n), int(mask)))

    def synchronize(self):
        self._check(lib().lbfd_synchronize(self._h))

    def read(self, field, comp=0):
        out = np.empty(self.N, np.float64)
        self._check(lib().lbfd_read(self._h, int(field), int(comp), out.ctypes.data_as(_dp)))
        return out.reshape(self.shape)

    def outlet_wave(self):
        """Characteristic outlet: incoming wave amplitude per outlet row [nz][ny]."""
        out = np.empty(self.N, np.float64)
        self._check(lib().lbfd_read(self._h, F_OUTLET_WAVE, 0, out.ctypes.data_as(_dp)))
        return out[: self.shape[0] * self.shape[1]].reshape(self.shape[:2]).copy()

    def set_outlet_wave(self, w):
        w = _f64(w)
        self._check(lib().lbfd_set_outlet_wave(self._h, w.ctypes.data_as(_dp)))

    def fields(self):
        d = {"rho": self.read(F_RHO), "T": self.read(F_T), "Ph": self.read(F_PH),
             "divu": self.read(F_DIVU)}
        d["u"] = np.stack([self.read(F_U, a) for a in range(self.dim)])
        if self.ns:
            d["Y"] = np.stack([self.read(F_Y, k) for k in range(self.ns)])
        return d

    def populations(self):
        return np.stack([self.read(F_POPULATIONS, i) for i in range(self.Q)])

    def diagnostics(self, allow_numeric=False):
        d = Diag()
        st = lib().lbfd_diagnostics(self._h, C.byref(d))
        if st != LBFD_OK and not (allow_numeric and st == LBFD_E_NUMERIC):
            self._check(st)
        out = {k: getattr(d, k) for k, _ in Diag._fields_
               if k not in ("species_mass", "n_fallback_reason")}
        out["species_mass"] = np.array(d.species_mass[: self.ns])
        out["n_fallback_reason"] = dict(zip(("envelope", "overdraw", "residual", "positivity"),
                                            list(d.n_fallback_reason)))
        out["status"] = st
        return out

    def bytes_per_cell(self):
        b = C.c_double()
        self._check(lib().lbfd_step_bytes_per_cell(self._h, C.byref(b)))
        return b.value

    # ------------------------------------------------------ surrogate
    def set_surrogate(self, weights, norm, envelope):
        """Install the chemistry surrogate (flat FP32 arrays in the ABI's
        layout), or remove it with weights=None."""
        if weights is None:
            self._check(lib().lbfd_set_surrogate(self._h, None, None, None))
            return
        fp = C.POINTER(C.c_float)
        arrs = [np.ascontiguousarray(np.asarray(a, np.float32)) for a in (weights, norm, envelope)]
        self._check(lib().lbfd_set_surrogate(self._h, *(a.ctypes.data_as(fp) for a in arrs)))

    def surrogate_eval(self, T, Y):
        """Surrogate on n states (torch float32 CUDA tensors T [n], Y [ns, n]):
        returns (raw [ns, n], omega [ns, n], fallback [n]) as CUDA tensors."""
        import torch

        T = T.contiguous().float()
        Y = Y.contiguous().float()
        n = T.numel()
        if Y.shape != (self.ns, n):
            raise ValueError("Y must be [ns, n]")
        raw = torch.empty((self.ns, n), dtype=torch.float32, device=T.device)
        om = torch.empty_like(raw)
        fb = torch.empty(n, dtype=torch.int32, device=T.device)
        self._check(lib().lbfd_surrogate_eval(self._h, T.data_ptr(), Y.data_ptr(), n,
                                              raw.data_ptr(), om.data_ptr(), fb.data_ptr()))
        self.synchronize()
        return raw, om, fb

    def sample_states(self, cells):
        """Training pairs at the given cells (int32 CUDA tensor of linear
        indices): x [n, 2 + ns] and the exact step source y [n, ns]."""
        import torch

        cells = cells.contiguous().to(torch.int32)
        n = cells.numel()
        x = torch.empty((n, 2 + self.ns), dtype=torch.float32, device=cells.device)
        y = torch.empty((n, self.ns), dtype=torch.float32, device=cells.device)
        self._check(lib().lbfd_sample_states(self._h, cells.data_ptr(), n, x.data_ptr(),
                                             y.data_ptr()))
        return x, y

    # ---------------------------------------------------- halo planes
    def halo_bytes(self):
        n = C.c_size_t()
        self._check(lib().lbfd_halo_bytes(self._h, C.byref(n)))
        return n.value

    def _halo_buf(self, buf):
        if not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("halo buffer must be a contiguous CUDA tensor")
        if buf.numel() * buf.element_size() < self.halo_bytes():
            raise ValueError("halo buffer too small")
        return buf.data_ptr()

    def halo_pack(self, face, buf):
        """Pack what the neighbour on `face` (-1 left, +1 right) needs for the
        next step into buf (populations for the state's AA parity, then T and
        Y_k of the own boundary plane)."""
        self._check(lib().lbfd_halo_pack(self._h, int(face), self._halo_buf(buf)))

    def halo_unpack(self, face, buf):
        """Unpack a buffer the neighbour on `face` packed for this slab."""
        self._check(lib().lbfd_halo_unpack(self._h, int(face), self._halo_buf(buf)))

    def set_timing(self, enable=True):
        self._check(lib().lbfd_set_timing(self._h, int(bool(enable))))

    def kernel_time(self, kernel=LBFD_KERNEL_STEP):
        """(timed launches, mean launch duration in ms) of one kernel kind."""
        n, ms = C.c_int64(), C.c_double()
        self._check(lib().lbfd_kernel_time(self._h, kernel, C.byref(n), C.byref(ms)))
        return n.value, ms.value


HIDDEN = 256


def surrogate_param_count(ns):
    ni = 2 + ns
    return HIDDEN * ni + HIDDEN + HIDDEN * HIDDEN + HIDDEN + ns * HIDDEN + ns


class Trainer:
    """Surrogate trainer on one GPU (owns a torch workspace and a C trainer).
    Data arrays are torch float32 CUDA tensors x [n, 2 + ns], y [n, ns]."""

    def __init__(self, n_species, batch=4096, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        L = lib()
        self.ns, self.batch = n_species, batch
        self.np = surrogate_param_count(n_species)
        self._cfg = TrainCfg(n_species, batch, beta1, beta2, eps)
        nbytes = C.c_size_t()
        st = L.lbfd_trainer_workspace_bytes(C.byref(self._cfg), C.byref(nbytes))
        if st != LBFD_OK:
            raise LbfdError(st, "trainer configuration")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = L.lbfd_trainer_create(C.byref(self._cfg), C.c_void_p(base + (-base) % 256),
                                   nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != LBFD_OK:
            raise LbfdError(st, "trainer create")
        self._h = h
        self._lib = L

    def _check(self, st):
        if st != LBFD_OK:
            raise LbfdError(st, lib().lbfd_trainer_last_error(self._h).decode())

    def __del__(self):
        h, L = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h and L is not None:
            L.lbfd_trainer_destroy(h)
            self._h = None

    def fit_norm(self, x, y):
        self._data = (x.contiguous(), y.contiguous())
        self._check(lib().lbfd_trainer_fit_norm(self._h, self._data[0].data_ptr(),
                                                self._data[1].data_ptr(), x.shape[0]))

    def set_weights(self, w):
        a = np.ascontiguousarray(np.asarray(w, np.float32))
        if a.size != self.np:
            raise ValueError(f"expected {self.np} weights")
        self._check(lib().lbfd_trainer_set_weights(self._h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def step(self, x, y, idx, lr, want_loss=False):
        loss = C.c_double()
        self._check(lib().lbfd_trainer_step(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                            idx.data_ptr(), float(lr),
                                            C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradient(self, x, y, idx):
        g = np.empty(self.np, np.float32)
        loss = C.c_double()
        self._check(lib().lbfd_trainer_gradient(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                                idx.data_ptr(), g.ctypes.data_as(C.POINTER(C.c_float)),
                                                C.byref(loss)))
        return g, loss.value

    def export(self):
        ni = 2 + self.ns
        w = np.empty(self.np, np.float32)
        nrm = np.empty(2 * ni + 2 * self.ns, np.float32)
        env = np.empty(2 * ni, np.float32)
        fp = C.POINTER(C.c_float)
        self._check(lib().lbfd_trainer_export(self._h, w.ctypes.data_as(fp), nrm.ctypes.data_as(fp),
                                              env.ctypes.data_as(fp)))
        return w, nrm, env

    def fit(self, x, y, epochs, lr, seed, lr_final=None, log=None):
        """Epochs of shuffled mini-batches; the permutations come from a seeded
        host generator and are passed to the device as batch indices.  The
        learning rate decays geometrically from lr to lr_final.  Returns the
        mean batch loss of each epoch."""
        import torch

        n = x.shape[0]
        rng = np.random.default_rng(seed)
        nb = n // self.batch
        total = max(1, epochs * nb)
        lr_final = lr if lr_final is None else lr_final
        out = []
        k = 0
        for e in range(epochs):
            perm = torch.tensor(rng.permutation(n)[: nb * self.batch].astype(np.int32),
                                device=x.device)
            losses = []
            for b in range(nb):
                rate = lr * (lr_final / lr) ** (k / total)
                last = b == nb - 1
                l = self.step(x, y, perm[b * self.batch:(b + 1) * self.batch], rate,
                              want_loss=(b % 16 == 0) or last)
                if l is not None:
                    losses.append(l)
                k += 1
            out.append(float(np.mean(losses)))
            if log:
                log(f"epoch {e}: loss {out[-1]:.4e}")
        return out
