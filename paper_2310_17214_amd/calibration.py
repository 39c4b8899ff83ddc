"""Calibration of the interface coupling constants A_u and A_T against the
sharp-interface (SI) reference (Sec. 4).

The diffuse-interface (DI) model adds a drag K = A_u mu phi_f phi_s^2/eta^2
(Eq. Fdrag-empirical-law) and a heat exchange H = A_T lambda phi_f
phi_s^2/eta^2 (Eq. diffusion-heat-flux-3).  Their constants are chosen so
that the DI solution in the bulk fluid comes closest to the SI one, run with
the coupling switched off and the phases separated at phi = 1/2.  The
distance between the two profiles across a channel section is the mean
standard error of Eq. mean-standard-error-f; a sweep of A_u (isothermal
flow, uniform inflow, Sec. 4.1) and of A_T (hot walls, fully developed
inflow, Sec. 4.2) locates the minimum.

Every simulation runs through the HIP library (lbfd.Context, FP64 mode);
this module only builds the channel inputs, reads the profiles and reduces
them.  Run as `python -m paper_2310_17214_amd.calibration` on a GPU host.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W


# ------------------------------------------------------------ the utility

def mse(f_si, f_di, x, L, eta):
    """Mean standard error of a DI profile against the SI one
    (Eq. mean-standard-error-f):

        MSE = 1/(L - eta) * int_{eta/2}^{L - eta/2} [(f_SI - f_DI)/f_SI,max]^2 dx

    over the bulk fluid of a channel of width L whose walls sit at x = 0 and
    x = L.  f_si, f_di: samples at the positions x (ascending; the channel's
    cell centres); f_SI,max is the largest |f_SI| of the samples.  The
    integrand is the square of the piecewise-linear interpolant of the
    normalised difference, integrated exactly (Simpson's rule is exact for
    the quadratic on each piece); the interval ends may fall between
    samples but must lie within [x[0], x[-1]]."""
    x = np.asarray(x, np.float64)
    f_si = np.asarray(f_si, np.float64)
    f_di = np.asarray(f_di, np.float64)
    a, b = 0.5 * eta, L - 0.5 * eta
    if not (b > a) or a < x[0] or b > x[-1] or np.any(np.diff(x) <= 0):
        raise ValueError("the bulk range [eta/2, L - eta/2] must lie inside the samples")
    fmax = np.max(np.abs(f_si))
    if not fmax > 0:
        raise ValueError("f_SI is zero everywhere")
    d = (f_si - f_di) / fmax
    # breakpoints: the samples inside (a, b) plus the two ends
    inner = x[(x > a) & (x < b)]
    pts = np.concatenate([[a], inner, [b]])
    dv = np.interp(pts, x, d)
    total = 0.0
    for i in range(len(pts) - 1):
        h = pts[i + 1] - pts[i]
        d0, d1 = dv[i], dv[i + 1]
        dm = 0.5 * (d0 + d1)
        total += h / 6.0 * (d0 * d0 + 4.0 * dm * dm + d1 * d1)
    return total / (L - eta)


def refine_minimum(values, errors):
    """The minimiser of a sampled MSE curve: the parabola in log(A) through
    the smallest sample and its two neighbours (the sample itself at an end
    of the sweep, where no bracket exists)."""
    v = np.asarray(values, np.float64)
    e = np.asarray(errors, np.float64)
    order = np.argsort(v)
    v, e = v[order], e[order]
    i = int(np.argmin(e))
    if i == 0 or i == len(v) - 1:
        return float(v[i]), False
    xs = np.log(v[i - 1:i + 2])
    ys = e[i - 1:i + 2]
    c2, c1, _ = np.polyfit(xs, ys, 2)
    if not c2 > 0:
        return float(v[i]), True
    xm = -c1 / (2.0 * c2)
    xm = min(max(xm, xs[0]), xs[2])
    return float(math.exp(xm)), True


# --------------------------------------------------------------- channel

def wall_profile(y, L, eta, shape="sine"):
    """Solid fraction across a channel whose walls sit at y = 0 and y = L:
    the larger of the two walls' profiles, each a function of the distance
    from its wall (Eq. def-phi: phi = (1 - sin(pi d/eta))/2 for |d| <= eta/2;
    `tanh`: the profile of the particle beds with the same centre and slope)."""
    prof = W.phase_sine if shape == "sine" else W.phase_tanh
    return np.maximum(prof(y, eta), prof(L - y, eta))


def channel(L=50, eta=8.0, H_over_L=5, Re=100.0, u0=0.04, thermal=False, T_wall=400.0,
            T_in=W.T_IN, si=False, A_u=W.A_U, A_T=70.0, shape="sine", precision="fp64"):
    """The calibration channel of Sec. 4 in the library's orientation: flow
    along x from a velocity inlet (-x) to the open, non-reflecting outlet
    (+x, the characteristic outlet with sigma = 0.25; a fixed-pressure outlet
    reflects the start-up pressure waves, which then slosh between inlet and
    outlet for longer than the flow takes to settle), the two
    walls across y at y = 0 and y = L (the wall lies half-way between the
    last solid and the first fluid cell centre, y_j = -eta/2 + j + 1/2).  The
    domain spans [-eta/2, L + eta/2] across the channel (the range the
    paper's profiles cover) and H = H_over_L L along it.

    Isothermal (Sec. 4.1): uniform inflow u0 over the fluid rows, walls and
    gas at T_in, constant viscosity.  Thermal (Sec. 4.2): the fully
    developed parabola with mean u0 over the fluid rows, walls at T_wall,
    inflow at T_in, Sutherland viscosity.  Re = L u0 / nu fixes nu.

    Returns (setup, phi, T0, inlet_profile, y) with y the rows' distances
    from the lower wall."""
    eta = float(eta)
    ny = int(round(L + eta))
    nx = int(round(H_over_L * L))
    s = W.base_setup(2, nx, ny, 1, 0, precision)
    s["lb_bc"] = ["inlet", "char_outlet", "wall", "wall", "periodic", "periodic"]
    s["outlet_sigma"] = 0.25
    s["fd_bc"] = ["dirichlet", "neumann", "dirichlet" if thermal else "neumann",
                  "dirichlet" if thermal else "neumann", "periodic", "periodic"]
    s["fd_val"][0] = [T_in]
    s["fd_val"][2] = [T_wall if thermal else T_in]
    s["fd_val"][3] = [T_wall if thermal else T_in]
    s["eta"] = eta
    s["T_in"] = T_in
    s["T_s"] = T_wall if thermal else T_in
    s["nu_in"] = u0 * L / Re
    s["mu_model"] = 1 if thermal else 0
    s["u_in"] = [u0, 0.0, 0.0]
    s["A_u"], s["A_T"] = float(A_u), float(A_T) if thermal else 0.0
    s["si"] = 1 if si else 0
    s["T_max"] = T_wall if thermal else 0.0
    y = -0.5 * eta + np.arange(ny) + 0.5
    phi_row = wall_profile(y, L, eta, shape)
    phi = np.broadcast_to(phi_row[None, :, None], (1, ny, nx)).copy()
    fluid = (y > 0) & (y < L)
    if thermal:
        xi = y / L
        uprof = np.where(fluid, 6.0 * u0 * xi * (1.0 - xi), 0.0)
    else:
        uprof = np.where(fluid, u0, 0.0)
    prof = np.zeros((2, 1, ny))
    prof[0, 0] = uprof
    # start: the gas at the inflow temperature, the solid at the wall's
    T0 = np.where(phi_row >= 0.5, s["T_s"], T_in) if si else (
        (1.0 - phi_row) * T_in + phi_row * s["T_s"])
    T0 = np.broadcast_to(T0[None, :, None], (1, ny, nx)).copy()
    return s, phi, T0, prof, y


def initial_velocity(prof, shape):
    """Start velocity: the inflow profile in every column (an impulsive start
    from rest sends a strong pressure wave through the channel)."""
    u0 = np.zeros((2,) + tuple(shape))
    u0[0] = prof[0][:, :, None]
    return u0


def run_channel(setup, phi, T0, prof, max_steps=200000, chunk=2000, tol=1e-7, section=0.9,
                log=None):
    """Step the channel on the GPU until the section profile settles: the
    largest change of u_x and T over `chunk` steps below tol (relative to
    their maxima).  Returns (u_x, T) across the section x = section H and the
    steps taken."""
    from . import lbfd

    ctx = lbfd.Context(setup, phi)
    ctx.set_inlet_profile(prof)
    ctx.init_state(T0, None, initial_velocity(prof, phi.shape))
    col = int(section * setup["nx"])
    prev = None
    steps = 0
    while steps < max_steps:
        ctx.step(chunk)
        steps += chunk
        f = ctx.fields()
        ux, T = f["u"][0][0, :, col].copy(), f["T"][0, :, col].copy()
        d = ctx.diagnostics()
        if d["n_nonfinite"]:
            raise RuntimeError("non-finite values in the channel run")
        if prev is not None:
            du = np.max(np.abs(ux - prev[0])) / max(np.max(np.abs(ux)), 1e-300)
            dT = np.max(np.abs(T - prev[1])) / max(np.max(np.abs(T)), 1e-300)
            if log:
                log(f"    step {steps}: change u {du:.2e} T {dT:.2e}")
            if du < tol and dT < tol:
                break
        prev = (ux, T)
    return ux, T, steps


def sweep(kind, values, eta, shape="sine", L=50, A_u_fixed=None, log=None, max_steps=200000,
          **kw):
    """MSE of the DI section profile against the SI one for each coupling
    value.  kind 'A_u': isothermal channel, f = u_x (Sec. 4.1); kind 'A_T':
    thermal channel, f = T (Sec. 4.2), with A_u at A_u_fixed."""
    thermal = kind == "A_T"
    base = dict(L=L, eta=eta, thermal=thermal, shape=shape, **kw)
    if thermal and A_u_fixed is not None:
        base["A_u"] = A_u_fixed
    s, phi, T0, prof, y = channel(si=True, **base)
    u_si, T_si, n_si = run_channel(s, phi, T0, prof, max_steps=max_steps)
    f_si = T_si if thermal else u_si
    fluid = (y > 0) & (y < L)
    out = {"kind": kind, "eta": eta, "shape": shape, "L": L, "si_steps": n_si, "runs": []}
    from . import lbfd

    for v in values:
        args = dict(base)
        args["A_T" if thermal else "A_u"] = v
        s, phi, T0, prof, _ = channel(si=False, **args)
        try:
            u_di, T_di, n = run_channel(s, phi, T0, prof, max_steps=max_steps)
        except lbfd.LbfdError as e:  # e.g. beyond the explicit-stability rule
            out["runs"].append({"value": float(v), "refused": str(e)})
            if log:
                log(f"  {kind} = {v:g}: refused ({e})")
            continue
        f_di = T_di if thermal else u_di
        e = mse(f_si[fluid], f_di[fluid], y[fluid], L, eta)
        out["runs"].append({"value": float(v), "mse": e, "steps": n})
        if log:
            log(f"  {kind} = {v:g}: MSE {e:.4e} ({n} steps)")
    ok = [r for r in out["runs"] if "mse" in r]
    vals = [r["value"] for r in ok]
    errs = [r["mse"] for r in ok]
    best, bracketed = refine_minimum(vals, errs)
    out["optimum"] = best
    out["bracketed"] = bracketed
    return out


def si_poiseuille(L=40, H_over_L=40, Re=100.0, u0=0.04, log=None):
    """Validation of the SI solver (Sec. 4.1): uniform inflow into a long
    channel (H = 40 L) between sharp walls; far downstream the profile must
    be the Poiseuille parabola 6 U xi (1 - xi), xi = y / L, with the walls
    half-way between the solid and the first fluid row.  Returns the
    largest deviation at x = 0.9 H relative to the parabola's maximum."""
    s, phi, T0, prof, y = channel(L=L, eta=2.0, H_over_L=H_over_L, Re=Re, u0=u0, si=True)
    ux, _, n = run_channel(s, phi, T0, prof, max_steps=400000, chunk=4000)
    fluid = (y > 0) & (y < L)
    xi = y[fluid] / L
    # mean velocity of the section (the inflow's, less the density change)
    U = ux[fluid].mean() / np.mean(6.0 * xi * (1.0 - xi))
    ref = 6.0 * U * xi * (1.0 - xi)
    return float(np.abs(ux[fluid] - ref).max() / ref.max()), n


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--eta", type=float, default=4.0)
    ap.add_argument("--shape", choices=["sine", "tanh"], default="tanh")
    ap.add_argument("--L", type=int, default=50)
    ap.add_argument("--A-u", type=float, nargs="*",
                    default=[40, 70, 100, 145, 200, 300, 450, 700, 1000, 1500, 2500, 4000,
                             7000])
    ap.add_argument("--A-T", type=float, nargs="*",
                    default=[20, 35, 50, 70, 100, 140, 200, 300, 450, 700, 1000, 1500])
    ap.add_argument("--poiseuille", action="store_true",
                    help="also validate the SI solver against the Poiseuille parabola")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    t0 = time.time()
    log(f"A_u sweep, eta = {a.eta}, {a.shape} profile, L = {a.L}")
    ru = sweep("A_u", a.A_u, a.eta, a.shape, a.L, log=log)
    log(f"A_u* = {ru['optimum']:.1f} (bracketed: {ru['bracketed']})")
    log(f"A_T sweep at A_u = {ru['optimum']:.1f}")
    rt = sweep("A_T", a.A_T, a.eta, a.shape, a.L, A_u_fixed=ru["optimum"], log=log)
    log(f"A_T* = {rt['optimum']:.1f} (bracketed: {rt['bracketed']})")
    res = {"command": "python -m paper_2310_17214_amd.calibration " + " ".join(argv or sys.argv[1:]),
           "A_u": ru, "A_T": rt}
    if a.poiseuille:
        err, n = si_poiseuille()
        log(f"SI Poiseuille (L = 40, H = 40 L, Re = 100): max deviation {err:.3e} "
            f"of the parabola's maximum after {n} steps")
        res["si_poiseuille"] = {"max_rel_dev": err, "steps": n}
    res["seconds"] = time.time() - t0
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
