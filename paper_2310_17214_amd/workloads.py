"""Seeded synthetic inputs for the coupled LB-FD-PF step.

This module produces *data only*: particle geometry turned into a solid phase
field, synthetic Arrhenius mechanism tables, physical parameters and initial
states.  It contains none of the method's arithmetic (no collision, transport
or reaction step) and imports neither the HIP binding nor the oracle, so both
sides can be fed identical inputs from it.

The paper's workloads (a methane/air two-step mechanism from a kinetics
library, an experimental cylinder bed, grain-growth particles) are not
available; seeded beds of spheres and superquadrics and generated mechanisms
with the same structure stand in for them.  Operating points follow the
paper: inlet at 300 K (Sec. 4.2), Sutherland constant S = 110.5 K (Eq. muT),
Pr = 0.7 (Sec. 4.2), A_u = 145 (Sec. 4.1) and A_T from the paper's fit
A_T* = 24.24 + 33.81 T_wall/T_inlet (Sec. 4.2).
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Optional

import numpy as np

LB_BC = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3, "char_outlet": 4}
FD_BC = {"periodic": 0, "dirichlet": 1, "neumann": 2}
MAX_SPECIES = 16
MAX_REACTIONS = 32

T_IN = 300.0
A_U = 145.0  # optimal momentum coupling, Sec. 4.1
THETA_IGN_BED = 1.0  # [K per step] FP64 reaction island threshold of the bed workloads


def a_t_fit(t_wall: float, t_inlet: float = T_IN) -> float:
    """Optimal heat-exchange coupling from the paper's linear fit (Sec. 4.2)."""
    return 24.24 + 33.81 * t_wall / t_inlet


# ----------------------------------------------------------------- geometry

def phase_tanh(d: np.ndarray, eta: float) -> np.ndarray:
    """Solid fraction from a signed distance d (> 0 in the fluid).

    The paper's profile is phi = (1 - sin(pi x/eta))/2 over one interface
    thickness (Eq. def-phi); the workloads ask for a tanh profile, taken with
    the same centre and the same slope at the centre."""
    return 0.5 * (1.0 - np.tanh(np.pi * d / eta))


def phase_sine(d: np.ndarray, eta: float) -> np.ndarray:
    """The paper's profile (Eq. def-phi), clamped to 0/1 outside |d| <= eta/2."""
    out = 0.5 * (1.0 - np.sin(np.pi * np.clip(d, -eta / 2, eta / 2) / eta))
    return out


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def cylinder_phi(nx: int, ny: int, cx: float, cy: float, r: float, eta: float) -> np.ndarray:
    """2-D disc (cell centre (i, j) at (i, j)); returns phi_s[1, ny, nx]."""
    x, y, _ = _grid((1, ny, nx))
    d = np.hypot(x - cx, y - cy) - r
    return phase_tanh(d, eta)


def _periodic_delta(a, b, length):
    d = a - b
    if length:
        d -= length * np.round(d / length)
    return d


def pack_spheres(n: int, r: float, box_lo, box_hi, periodic, seed: int,
                 iters: int = 4000, margin: float = 1e-3) -> np.ndarray:
    """Random non-overlapping sphere centres by collective rearrangement.

    Centres start uniform in the box and overlapping pairs are pushed apart
    symmetrically until no pair is closer than 2r (periodic axes use the
    minimum image; non-periodic axes clamp centres into the box)."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    lo = np.asarray(box_lo, float)
    hi = np.asarray(box_hi, float)
    L = hi - lo
    per = np.asarray(periodic, bool)
    p = lo + rng.random((n, 3)) * L
    big = 1e9
    boxsize = np.where(per, L, big)
    for _ in range(iters):
        q = p - lo
        q = np.where(per, np.mod(q, L), q + big / 2)
        tree = cKDTree(q, boxsize=boxsize)
        pairs = tree.query_pairs(2.0 * r, output_type="ndarray")
        if len(pairs) == 0:
            break
        i, j = pairs[:, 0], pairs[:, 1]
        d = p[i] - p[j]
        for a in range(3):
            if per[a]:
                d[:, a] -= L[a] * np.round(d[:, a] / L[a])
        dist = np.linalg.norm(d, axis=1)
        dist = np.maximum(dist, 1e-9)
        push = (2.0 * r - dist + margin) / 2.0
        step = d / dist[:, None] * push[:, None]
        np.add.at(p, i, step)
        np.add.at(p, j, -step)
        for a in range(3):
            if per[a]:
                p[:, a] = lo[a] + np.mod(p[:, a] - lo[a], L[a])
            else:
                p[:, a] = np.clip(p[:, a], lo[a], hi[a])
    return p


def _rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


@dataclasses.dataclass
class Particle:
    centre: np.ndarray
    kind: str = "sphere"            # "sphere" | "superquadric"
    r: float = 8.0                  # sphere radius / equivalent radius
    axes: Optional[np.ndarray] = None
    expo: float = 2.0
    rot: Optional[np.ndarray] = None


def particle_distance(p: Particle, x, y, z, shape, periodic) -> np.ndarray:
    """Approximate signed distance (> 0 outside) of a particle, evaluated on a
    set of points; exact for spheres, d ~ r_eq (F^(1/n) - 1) for superquadrics."""
    nz, ny, nx = shape
    dx = _periodic_delta(x, p.centre[0], nx if periodic[0] else 0)
    dy = _periodic_delta(y, p.centre[1], ny if periodic[1] else 0)
    dz = _periodic_delta(z, p.centre[2], nz if periodic[2] else 0)
    if p.kind == "sphere":
        return np.sqrt(dx * dx + dy * dy + dz * dz) - p.r
    R = p.rot
    bx = R[0, 0] * dx + R[1, 0] * dy + R[2, 0] * dz
    by = R[0, 1] * dx + R[1, 1] * dy + R[2, 1] * dz
    bz = R[0, 2] * dx + R[1, 2] * dy + R[2, 2] * dz
    n = p.expo
    F = (np.abs(bx / p.axes[0]) ** n + np.abs(by / p.axes[1]) ** n + np.abs(bz / p.axes[2]) ** n)
    return p.r * (F ** (1.0 / n) - 1.0)


def _particle_box(p: Particle, shape, eta: float, periodic):
    """Cell index lists (x, y, z) of the box a particle's phase field reaches."""
    nz, ny, nx = shape
    reach = 2.0 * eta + 1.0
    ext = (p.r * (float(np.max(p.axes)) / p.r if p.axes is not None else 1.0)) + reach
    ext = max(ext, p.r * 1.6 + reach) if p.kind == "superquadric" else ext
    idx = []
    for a, n in enumerate((nx, ny, nz)):
        lo = int(math.floor(p.centre[a] - ext))
        hi = int(math.ceil(p.centre[a] + ext)) + 1
        rng_ = np.arange(lo, hi)
        if periodic[a]:
            rng_ = np.mod(rng_, n)
            rng_ = np.unique(rng_)
        else:
            rng_ = rng_[(rng_ >= 0) & (rng_ < n)]
        idx.append(rng_)
    return idx


def _bed_phi_planes(shape, particles, eta, periodic, z0, z1):
    """Planes z0 <= z < z1 of bed_phi (max over the particles reaching them)."""
    nz, ny, nx = shape
    phi = np.zeros((z1 - z0, ny, nx), np.float64)
    for p in particles:
        ix, iy, iz = _particle_box(p, shape, eta, periodic)
        iz = iz[(iz >= z0) & (iz < z1)]
        if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
            continue
        zz, yy, xx = np.meshgrid(iz, iy, ix, indexing="ij")
        d = particle_distance(p, xx.astype(float), yy.astype(float), zz.astype(float), shape,
                              periodic)
        ph = phase_tanh(d, eta)
        sel = np.ix_(iz - z0, iy, ix)
        phi[sel] = np.maximum(phi[sel], ph)
    return phi


def bed_phi(shape, particles, eta: float, periodic, workers=None) -> np.ndarray:
    """Union (max) of the particles' tanh phase fields on a [nz, ny, nx] grid.

    Large grids are computed in z-slabs by a pool of processes; each cell's
    value is the same maximum of the same per-particle values either way."""
    import os

    nz, ny, nx = shape
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if nz * ny * nx >= (1 << 23) else 1
    if workers <= 1 or nz < 2 * workers:
        return _bed_phi_planes(shape, particles, eta, periodic, 0, nz)
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    bounds = np.linspace(0, nz, workers + 1).astype(int)
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        parts = list(ex.map(_bed_phi_planes, [shape] * workers, [particles] * workers,
                            [eta] * workers, [periodic] * workers, bounds[:-1], bounds[1:]))
    return np.concatenate(parts, axis=0)


def sharp_solid(shape, particles, periodic) -> np.ndarray:
    """Voxelised sharp geometry (cell centre inside any particle)."""
    nz, ny, nx = shape
    solid = np.zeros(shape, bool)
    for p in particles:
        ext = p.r * 1.8 + 1.0
        idx = []
        for a, n in enumerate((nx, ny, nz)):
            rng_ = np.arange(int(math.floor(p.centre[a] - ext)), int(math.ceil(p.centre[a] + ext)) + 1)
            rng_ = np.unique(np.mod(rng_, n)) if periodic[a] else rng_[(rng_ >= 0) & (rng_ < n)]
            idx.append(rng_)
        if any(len(i) == 0 for i in idx):
            continue
        zz, yy, xx = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
        d = particle_distance(p, xx.astype(float), yy.astype(float), zz.astype(float), shape,
                              periodic)
        sub = solid[np.ix_(idx[2], idx[1], idx[0])]
        solid[np.ix_(idx[2], idx[1], idx[0])] = sub | (d <= 0)
    return solid


def sphere_bed(shape, x_range, r, porosity, seed, periodic=(False, True, True), n=None):
    """Dense random bed of equal spheres filling x in [x0, x1) at a target
    porosity measured on the sharp geometry inside the bed region."""
    nz, ny, nx = shape
    x0, x1 = x_range
    vol = (x1 - x0) * ny * nz
    if n is None:
        n = int(round((1.0 - porosity) * vol / (4.0 / 3.0 * math.pi * r ** 3)))
    lo = (x0 + 0.5 * r, 0.0, 0.0)
    hi = (x1 - 0.5 * r, float(ny), float(nz))
    centres = pack_spheres(n, r, lo, hi, (False, periodic[1], periodic[2]), seed)
    return [Particle(centre=c, kind="sphere", r=r) for c in centres]


def superquadric_bed(shape, x_range, r_eq, porosity, seed, sphere_share=0.0,
                     periodic=(False, True, True)):
    """Bed of randomly oriented superquadrics (one exponent n ~ U[2, 8] per
    particle, aspect ratios ~ U[0.75, 1.33] normalised to equal volume with a
    sphere of radius r_eq); a share of plain spheres may be mixed in.
    Centres are placed by the sphere packer on equivalent spheres; particles
    may touch where their shapes stick out of the equivalent sphere."""
    rng = np.random.default_rng(seed + 1000)
    base = sphere_bed(shape, x_range, r_eq, porosity, seed, periodic)
    out = []
    for p in base:
        if rng.random() < sphere_share:
            out.append(p)
            continue
        ar = rng.uniform(0.75, 1.33, size=3)
        ar /= np.prod(ar) ** (1.0 / 3.0)
        n = float(rng.uniform(2.0, 8.0))
        # volume of |x|^n+|y|^n+|z|^n <= 1 is 8 G(1+1/n)^3 / G(1+3/n)
        unit = 8.0 * math.gamma(1 + 1 / n) ** 3 / math.gamma(1 + 3 / n)
        scale = (4.0 / 3.0 * math.pi / unit) ** (1.0 / 3.0) * r_eq
        out.append(Particle(centre=p.centre, kind="superquadric", r=r_eq, axes=ar * scale,
                            expo=n, rot=_rotation(rng)))
    return out


def bed_porosity(solid: np.ndarray, x_range) -> float:
    x0, x1 = x_range
    return 1.0 - float(solid[:, :, x0:x1].mean())


# ---------------------------------------------------------------- mechanisms

def mech_empty(ns: int):
    return dict(M=[1.0] * ns, dhf=[0.0] * ns, mu_star=[1.0] * ns,
                nu_f=[], nu_r=[], A=[], beta=[], theta=[], rev=[], lnKc_a=[], lnKc_b=[])


def mech_one_step(theta=15000.0, q_over_cp=2000.0, A=1.0):
    """Irreversible F + O -> 2P with inert N, all molar masses 1 (so rho ~ 1/T).
    Species order: F, O, P, N.  Formation enthalpies per unit mass, in units
    of cp*K: only the fuel carries chemical enthalpy, Q/cp = 2000 K."""
    return dict(M=[1.0, 1.0, 1.0, 1.0], dhf=[q_over_cp, 0.0, 0.0, 0.0], mu_star=[1.0] * 4,
                nu_f=[[1, 1, 0, 0]], nu_r=[[0, 0, 2, 0]], A=[A], beta=[0.0], theta=[theta],
                rev=[0], lnKc_a=[0.0], lnKc_b=[0.0])


# Pseudo-elements (a, b, d) with integer masses; d only in the inert diluent.
_ELEM_MASS = np.array([1, 16, 28])
_SPECIES = [  # element vectors of the 9 synthetic species (last = inert diluent)
    (2, 0, 0), (0, 2, 0), (2, 1, 0), (1, 1, 0), (1, 0, 0),
    (0, 1, 0), (1, 2, 0), (2, 2, 0), (0, 0, 1)]
SYNTH9_NAMES = ["A2", "B2", "A2B", "AB", "A", "B", "AB2", "A2B2", "D"]


def _balanced_candidates(nreact: int):
    comp = np.array(_SPECIES[:nreact])
    cands = []
    idx = range(nreact)
    for a, b in itertools.combinations_with_replacement(idx, 2):
        lhs = comp[a] + comp[b]
        for c, d in itertools.combinations_with_replacement(idx, 2):
            if {a, b} & {c, d}:
                continue
            if np.array_equal(lhs, comp[c] + comp[d]) and (a, b) < (c, d):
                cands.append(((a, b), (c, d)))
        for c in idx:
            if c in (a, b):
                continue
            if np.array_equal(lhs, comp[c]):
                cands.append(((a, b), (c,)))
    return cands


def mech_synthetic9(seed=33, nr=21, T_ref=1500.0, conc_ref=None, n_sub_target=8,
                    cp=1.0, R_over_M_in=0.2857):
    """Synthetic 9-species, 21-reversible-reaction mechanism.

    Mass balance is exact: species are small integer vectors over pseudo-
    elements and every reaction is drawn from the element-balanced candidates
    of the forms A+B=C+D, A+B=C (and their reverse A=B+C).  Rate parameters
    are seeded in realistic ranges (theta ~ U[0, 20000] K, beta ~ U[-1, 1],
    A log-uniform over three decades) and then scaled together so that a
    pseudo-first-order rate bound at T_ref and the reference concentrations
    gives h*kappa <= 0.5 with n_sub_target sub-steps.  Equilibrium constants
    are thermodynamically consistent: ln Kc = a + b/T with b = -dH/R from the
    same formation-enthalpy table (dH is the molar reaction enthalpy) and
    a = sum_k s_kj sigma_k + dn_j ln(c0) from seeded species constants
    sigma_k ~ U[-1, 1] and a standard-state concentration c0 = 1e-4."""
    rng = np.random.default_rng(seed)
    ns = 9
    comp = np.array(_SPECIES)
    M = (comp @ _ELEM_MASS).astype(float)
    cands = _balanced_candidates(8)
    # initiation from the fresh mixture (A2 + B2) is always present; the rest
    # are drawn from the remaining candidates
    init = [i for i, (lhs, _) in enumerate(cands) if sorted(lhs) == [0, 1]]
    rest = [i for i in range(len(cands)) if i not in init]
    pick = np.concatenate([init, rng.choice(rest, size=nr - len(init), replace=False)])
    nu_f = np.zeros((nr, ns), int)
    nu_r = np.zeros((nr, ns), int)
    for j, ci in enumerate(sorted(pick)):
        lhs, rhs = cands[ci]
        if rng.random() < 0.3 and len(rhs) == 1:  # write as dissociation A = B + C
            lhs, rhs = rhs, lhs
        for s in lhs:
            nu_f[j, s] += 1
        for s in rhs:
            nu_r[j, s] += 1
    # formation enthalpy per unit mass (units cp*K): fuels and radicals positive,
    # products negative, diluent zero; "fuel-like -> product" is exothermic.
    dhf = np.array([0.0, 0.0, -3000.0, 2000.0, 30000.0, 4000.0, 100.0, -1000.0, 0.0])
    dH = (nu_r - nu_f) @ (dhf * M)           # molar reaction enthalpy (cp*K*mass/mol)
    R_u = R_over_M_in * _mbar_in_synth9()    # gas constant in the same units
    lnKc_b = -dH / R_u
    # entropy-like species constants: ln Kc_j = sum_k s_kj (sigma_k - h_k/(R T)),
    # so the equilibrium constants are consistent around every reaction cycle
    # plus dn_j ln(c0) for a standard-state concentration c0 typical of the
    # lattice-unit concentrations (reactions changing the mole count)
    sigma = rng.uniform(-1.0, 1.0, ns)
    dn = (nu_r - nu_f).sum(axis=1)
    lnKc_a = (nu_r - nu_f) @ sigma + dn * math.log(1e-4)
    theta = rng.uniform(0.0, 20000.0, nr)
    beta = rng.uniform(-1.0, 1.0, nr)
    yref = np.maximum(np.maximum(SYNTH9_Y_IN, burnt_synth9()), 0.01)

    def kappa(Avec, T):
        """Pseudo-first-order consumption rate of each species at temperature T
        (concentrations rho Y/M with rho ~ T_in/T, the larger of the inlet and
        burnt fractions, at least 1 %), and the largest per-reaction term."""
        conc = (T_IN / T) * yref / M if conc_ref is None else conc_ref
        kf = Avec * T ** beta * np.exp(-theta / T)
        kr = kf / np.exp(lnKc_a + lnKc_b / T)
        kap = np.zeros(ns)
        per = np.zeros(nr)
        for j in range(nr):
            for nu, kk in ((nu_f[j], kf[j]), (nu_r[j], kr[j])):
                for k in range(ns):
                    if nu[k] == 0:
                        continue
                    other = kk
                    for m_ in range(ns):
                        e = nu[m_] - (1 if m_ == k else 0)
                        other *= conc[m_] ** e
                    kap[k] += nu[k] * other
                    per[j] = max(per[j], nu[k] * other)
        return kap, per

    # each reaction normalised by its largest rate over T_in..T_ref, then
    # spread log-uniformly over three decades below a common target rate; the
    # stiffness bound over the same range fixes n_sub (h kappa <= 0.5, at most
    # 32 sub-steps, A scaled down if needed)
    temps = np.linspace(T_IN, T_ref, 18)
    per = np.max([kappa(np.ones(nr), T)[1] for T in temps], axis=0)
    target = 0.5 * n_sub_target / 4.0
    A = 10.0 ** rng.uniform(-3.0, 0.0, nr) * target / per
    kmax = max(float(kappa(A, T)[0].max()) for T in temps)
    if kmax > 0.5 * 32:
        A *= 0.5 * 32 / kmax
        kmax = 0.5 * 32
    n_sub = int(min(32, max(1, math.ceil(kmax / 0.5))))
    return dict(M=M.tolist(), dhf=dhf.tolist(), mu_star=rng.uniform(0.7, 1.4, ns).tolist(),
                nu_f=nu_f.tolist(), nu_r=nu_r.tolist(), A=A.tolist(), beta=beta.tolist(),
                theta=theta.tolist(), rev=[1] * nr, lnKc_a=lnKc_a.tolist(),
                lnKc_b=lnKc_b.tolist(), n_sub=n_sub)


SYNTH9_Y_IN = [0.03, 0.30, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.67]


def _mbar_in_synth9():
    comp = np.array(_SPECIES)
    M = comp @ _ELEM_MASS
    y = np.array(SYNTH9_Y_IN)
    return 1.0 / float(np.sum(y / M))


def burnt_synth9():
    """Products of the synthetic inlet mixture (all A2 burnt to A2B with B2):
    mass fractions that conserve every pseudo-element of SYNTH9_Y_IN."""
    comp = np.array(_SPECIES, float)
    M = comp @ _ELEM_MASS
    yin = np.array(SYNTH9_Y_IN)
    elem_in = (yin / M) @ comp                   # moles of each element per unit mass
    n_a2b = elem_in[0] / 2.0
    n_b2 = (elem_in[1] - n_a2b) / 2.0
    y = np.zeros(9)
    y[2] = n_a2b * M[2]
    y[1] = n_b2 * M[1]
    y[8] = elem_in[2] * M[8]
    return (y / y.sum()).tolist()


# ------------------------------------------------------------------ configs

def _faces(kind_x0, kind_x1, kind_y, kind_z):
    return [kind_x0, kind_x1, kind_y, kind_y, kind_z, kind_z]


@dataclasses.dataclass
class Workload:
    name: str
    setup: dict
    phi: np.ndarray          # [nz, ny, nx] solid fraction
    T0: np.ndarray           # [nz, ny, nx]
    Y0: np.ndarray           # [ns, nz, ny, nx]
    u0: Optional[np.ndarray]  # [dim, nz, ny, nx] or None
    steps: int
    notes: str = ""

    @property
    def cells(self) -> int:
        s = self.setup
        return s["nx"] * s["ny"] * s["nz"]


def base_setup(dim, nx, ny, nz, ns, precision="fp64"):
    return dict(
        dim=dim, nx=nx, ny=ny, nz=nz, ns=ns, precision=precision,
        lb_bc=["periodic"] * 6, fd_bc=["periodic"] * 6,
        fd_val=[[0.0] * (1 + ns) for _ in range(6)],
        A_u=A_U, A_T=0.0, eta=4.0, T_s=T_IN, Pr=0.7, cp=1.0, rho_in=1.0, T_in=T_IN,
        nu_in=0.02, S_suth=110.5, mu_model=1, transport=0,
        u_in=[0.0, 0.0, 0.0], F_b=[0.0, 0.0, 0.0], Y_in=[1.0 / max(ns, 1)] * ns,
        Le=[1.0] * ns, n_sub=1, theta_ign=1e-6, mech=mech_empty(ns))


def cylinder_channel() -> Workload:
    """2-D D2Q9 channel 128x64, FP64: one solid cylinder r = 10 at (32, 32),
    tanh phase field of width 4, inert gas, inlet u = 0.02, Re = 20 on the
    diameter (nu = 0.02), cylinder held at 1.5 T_inlet, Pr = 0.7, 2000 steps."""
    nx, ny = 128, 64
    s = base_setup(2, nx, ny, 1, 0, "fp64")
    s["lb_bc"] = _faces("inlet", "outlet", "wall", "periodic")
    s["fd_bc"] = _faces("dirichlet", "neumann", "neumann", "periodic")
    s["fd_val"][0] = [T_IN]
    s["u_in"] = [0.02, 0.0, 0.0]
    s["nu_in"] = 0.02 * 20.0 / 20.0
    s["T_s"] = 1.5 * T_IN
    s["A_T"] = a_t_fit(s["T_s"])
    phi = cylinder_phi(nx, ny, 32.0, 32.0, 10.0, s["eta"])
    T0 = (1.0 - phi) * T_IN + phi * s["T_s"]
    return Workload("cylinder_channel_d2q9_128x64", s, phi, T0, np.zeros((0, 1, ny, nx)), None,
                    2000)


def _reactive_bed_setup(dim, nx, ny, nz, mech, Y_in, precision, T_s, nu_in, u_in, transport,
                        Le, n_sub):
    ns = len(Y_in)
    s = base_setup(dim, nx, ny, nz, ns, precision)
    s["lb_bc"] = _faces("inlet", "outlet", "periodic", "periodic")
    s["fd_bc"] = _faces("dirichlet", "neumann", "periodic", "periodic")
    s["fd_val"][0] = [T_IN] + list(Y_in)
    s["u_in"] = [u_in, 0.0, 0.0]
    s["nu_in"] = nu_in
    s["T_s"] = T_s
    s["A_T"] = a_t_fit(T_s)
    s["Y_in"] = list(Y_in)
    s["Le"] = list(Le)
    s["transport"] = transport
    s["n_sub"] = n_sub
    s["mech"] = mech
    # FP32 mode: cells releasing more than 1 K of heat per step (actively
    # burning, where the reaction sub-steps are stiff) integrate them in FP64
    s["theta_ign"] = THETA_IGN_BED
    return s


def one_step_rate_constant(t_ad=1100.0, theta=15000.0, rho_ad=T_IN / 1100.0, y_o=0.5,
                           tau_steps=50.0):
    """Pre-exponential factor so that 1/(A exp(-theta/T_ad) rho_ad Y_O) = tau_steps."""
    return 1.0 / (tau_steps * math.exp(-theta / t_ad) * rho_ad * y_o)


ONE_STEP_Y_IN = [0.4, 0.5, 0.0, 0.1]
ONE_STEP_Y_BURNT = [0.0, 0.1, 0.8, 0.1]


def _split_init(shape, phi, x_split, T_fresh, Y_fresh, T_burnt, Y_burnt, T_s):
    nz, ny, nx = shape
    x = np.arange(nx)[None, None, :]
    burnt = np.broadcast_to(x >= x_split, shape)
    Tg = np.where(burnt, T_burnt, T_fresh)
    T0 = (1.0 - phi) * Tg + phi * T_s
    ns = len(Y_fresh)
    Y0 = np.empty((ns,) + shape)
    for k in range(ns):
        Y0[k] = np.where(burnt, Y_burnt[k], Y_fresh[k])
    return T0, Y0


def bed_one_step(nx=256, ny=128, nz=128, precision="fp32", seed=2, bed=(32, 224), x_split=96,
             porosity=0.40, r=8.0, steps=5000) -> Workload:
    """3-D D3Q19 packed channel (default 256x128x128), seeded random spheres
    r = 8 at porosity 0.4, tanh width 4, rho ~ 1/T, one-step irreversible
    F + O -> 2P with theta = 15000 K and Q/cp = 2000 K, lean premixed inlet."""
    mech = mech_one_step(A=one_step_rate_constant())
    s = _reactive_bed_setup(3, nx, ny, nz, mech, ONE_STEP_Y_IN, precision, T_s=700.0, nu_in=0.008,
                            u_in=0.005, transport=0, Le=[1.0] * 4, n_sub=1)
    shape = (nz, ny, nx)
    parts = sphere_bed(shape, bed, r, porosity, seed)
    phi = bed_phi(shape, parts, s["eta"], (False, True, True))
    T0, Y0 = _split_init(shape, phi, x_split, T_IN, ONE_STEP_Y_IN, 1100.0, ONE_STEP_Y_BURNT, s["T_s"])
    wl = Workload(f"sphere_bed_one_step_d3q19_{nx}x{ny}x{nz}", s, phi, T0, Y0, None, steps)
    wl.particles = parts
    wl.bed = bed
    return wl


def bed_superquadric_9sp(nx=384, ny=192, nz=192, precision="fp32", seed=3, bed=(48, 336), x_split=144,
             porosity=0.45, steps=5000, sphere_share=0.0, mech_seed=33,
             T_burnt=1100.0) -> Workload:
    """3-D D3Q19 bed of seeded superquadrics, synthetic 9-species /
    21-reversible-reaction mechanism, Wilke mixture transport with constant
    Lewis numbers ~ U[0.8, 1.2], FP32 fields with FP64 reaction sub-steps."""
    mech = mech_synthetic9(seed=mech_seed)
    rng = np.random.default_rng(seed + 77)
    Le = rng.uniform(0.8, 1.2, 9).tolist()
    Le[8] = 1.0
    s = _reactive_bed_setup(3, nx, ny, nz, mech, SYNTH9_Y_IN, precision, T_s=700.0,
                            nu_in=0.006, u_in=0.005, transport=1, Le=Le,
                            n_sub=int(mech["n_sub"]))
    shape = (nz, ny, nx)
    parts = superquadric_bed(shape, bed, 8.0, porosity, seed, sphere_share=sphere_share)
    phi = bed_phi(shape, parts, s["eta"], (False, True, True))
    T0, Y0 = _split_init(shape, phi, x_split, T_IN, SYNTH9_Y_IN, T_burnt, burnt_synth9(),
                         s["T_s"])
    wl = Workload(f"superquadric_bed_9species_d3q19_{nx}x{ny}x{nz}", s, phi, T0, Y0, None, steps)
    wl.particles = parts
    wl.bed = bed
    return wl


def bed_sphere_9sp(nx=256, ny=128, nz=128, precision="fp32", seed=2, bed=(32, 224), x_split=96,
             porosity=0.40, r=8.0, steps=5000, mech_seed=33, T_burnt=1100.0) -> Workload:
    """The sphere bed of bed_one_step (grid, particles, flow, heat exchange) with the
    synthetic 9-species / 21-reversible-reaction mechanism: the workload of
    the chemistry surrogate."""
    mech = mech_synthetic9(seed=mech_seed)
    s = _reactive_bed_setup(3, nx, ny, nz, mech, SYNTH9_Y_IN, precision, T_s=700.0,
                            nu_in=0.008, u_in=0.005, transport=0, Le=[1.0] * 9,
                            n_sub=int(mech["n_sub"]))
    shape = (nz, ny, nx)
    parts = sphere_bed(shape, bed, r, porosity, seed)
    phi = bed_phi(shape, parts, s["eta"], (False, True, True))
    T0, Y0 = _split_init(shape, phi, x_split, T_IN, SYNTH9_Y_IN, T_burnt, burnt_synth9(),
                         s["T_s"])
    wl = Workload(f"sphere_bed_9species_d3q19_{nx}x{ny}x{nz}", s, phi, T0, Y0, None, steps)
    wl.particles = parts
    wl.bed = bed
    return wl


def bed_elongated_9sp(nx=1024, ny=256, nz=256, precision="fp32", seed=5, bed=(64, 960),
                      x_split=352, porosity=0.40, sphere_share=0.5, steps=20000, window=None,
                      mech_seed=33, T_burnt=1100.0, log=None) -> Workload:
    """3-D D3Q19 elongated bed (default 1024x256x256) of seeded particles, half
    spheres and half superquadrics (r_eq = 8, porosity 0.4), with the
    9-species mechanism and the mixture transport of bed_superquadric_9sp.

    window=(x0, x1) builds only the cells x0 <= x < x1 of that bed: the share
    of one GPU in a decomposition into slabs along x, with one halo plane on
    each side (e.g. (255, 385) for the third of eight 128-cell slabs).  Its
    x faces keep the inlet and outlet rules; in a decomposed run the halo
    exchange overwrites them."""
    mech = mech_synthetic9(seed=mech_seed)
    rng = np.random.default_rng(seed + 77)
    Le = rng.uniform(0.8, 1.2, 9).tolist()
    Le[8] = 1.0
    x0, x1 = (0, nx) if window is None else window
    if not 0 <= x0 < x1 <= nx:
        raise ValueError("window outside the bed")
    wx = x1 - x0
    s = _reactive_bed_setup(3, wx, ny, nz, mech, SYNTH9_Y_IN, precision, T_s=700.0,
                            nu_in=0.006, u_in=0.005, transport=1, Le=Le,
                            n_sub=int(mech["n_sub"]))
    parts = superquadric_bed((nz, ny, nx), bed, 8.0, porosity, seed, sphere_share=sphere_share)
    if log:
        log(f"placed {len(parts)} particles")
    if window is not None:
        reach = 8.0 * 1.6 + 2.0 * s["eta"] + 2.0
        parts = [dataclasses.replace(p, centre=p.centre - np.array([x0, 0.0, 0.0]))
                 for p in parts if x0 - reach <= p.centre[0] < x1 + reach]
    shape = (nz, ny, wx)
    phi = bed_phi(shape, parts, s["eta"], (False, True, True))
    if log:
        log("phase field done")
    T0, Y0 = _split_init(shape, phi, x_split - x0, T_IN, SYNTH9_Y_IN, T_burnt, burnt_synth9(),
                         s["T_s"])
    name = f"elongated_bed_9species_d3q19_{nx}x{ny}x{nz}"
    if window is not None:
        name += f"_slab_x{x0}-{x1}"
    wl = Workload(name, s, phi, T0, Y0, None, steps)
    wl.particles = parts
    wl.bed = (bed[0] - x0, bed[1] - x0)
    return wl


# ----------------------------------------------------- small test setups

def periodic_box(dim, n, ns=0, precision="fp64"):
    nz = n if dim == 3 else 1
    return base_setup(dim, n, n, nz, ns, precision)


def random_smooth_field(shape, seed, amp=1.0, modes=3):
    """Smooth periodic random field (sum of a few low Fourier modes)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    f = np.zeros(shape)
    for _ in range(modes):
        kx, ky, kz = rng.integers(0, 3, 3)
        ph = rng.uniform(0, 2 * np.pi)
        f += rng.normal() * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / max(nz, 1))
                                   + ph)
    return amp * f / max(1.0, np.abs(f).max())
