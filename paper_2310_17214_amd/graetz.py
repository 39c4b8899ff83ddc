"""Thermal entrance of plug flow between isothermal walls (Sec. 4.3): the
paper's Graetz-type series and a grid-convergence study of the FD
temperature transport against it.

Flow along x at a uniform velocity U between two walls at y = 0 and y = L
held at T_w; the gas enters at T_in.  Without axial conduction the steady
temperature is the series of Eq. graetz_solution,

    T^(x, y) = (T - T_w)/(T_in - T_w)
             = sum_{n odd} 4/(n pi) sin(n pi y/L) exp(-(n pi/L)^2 alpha x/U),

(as printed it is the plug-flow solution; with a parabolic profile the
eigenfunctions differ).

In the library the channel is a D2Q9 grid whose y faces are periodic for the
flow (so the flow stays uniform) and Dirichlet at T_w for the temperature
(cell-centred ghosts: the walls sit on the ghost centres, L = ny + 1); the
inlet face holds T_in on its ghost (x = 0 one cell before the first column).
The steady FD equations -- first-order upwind convection, central diffusion
-- then have an exact discrete solution: discrete sine modes across the
channel, each decaying geometrically along x,

    T^_ij = sum_n b_n sin(n pi y_j / L) r_n^(i + 1),
    alpha r^2 - (2 alpha + alpha kappa_n + U) r + (alpha + U) = 0,  |r_n| < 1,
    kappa_n = 2 - 2 cos(n pi / L),

with b_n the discrete sine coefficients of the uniform inflow (the upwind
scheme adds a numerical diffusion U/2 along x; the time step does not enter
the steady state).  `discrete_solution` evaluates it; the GPU steady state
must match it to the flow's own small non-uniformity, and the convergence
study measures how fast the scheme approaches the continuous series.
"""
import argparse
import json
import math
import sys

import numpy as np

from . import workloads as W


def series(x, y, L, alpha, U, nterms=401):
    """The plug-flow series of Eq. graetz_solution (no axial conduction)."""
    x = np.asarray(x, float)[..., None]
    y = np.asarray(y, float)[..., None]
    n = np.arange(1, 2 * nterms, 2, dtype=float)
    k = n * math.pi / L
    return np.sum(4.0 / (n * math.pi) * np.sin(k * y) * np.exp(-k * k * alpha * x / U), axis=-1)


def series_axial(x, y, L, alpha, U, nterms=401):
    """The same entrance problem with axial conduction kept (the PDE
    U dT/dx = alpha (d2T/dx2 + d2T/dy2) for x > 0, T(0, y) = T_in, bounded
    downstream): each sine mode decays as exp(mu_n x) with
    mu_n = (U - sqrt(U^2 + 4 alpha^2 k_n^2)) / (2 alpha), k_n = n pi / L; it
    tends to the series above as the Peclet number grows."""
    x = np.asarray(x, float)[..., None]
    y = np.asarray(y, float)[..., None]
    n = np.arange(1, 2 * nterms, 2, dtype=float)
    k = n * math.pi / L
    mu = (U - np.sqrt(U * U + 4.0 * alpha * alpha * k * k)) / (2.0 * alpha)
    return np.sum(4.0 / (n * math.pi) * np.sin(k * y) * np.exp(mu * x), axis=-1)


def discrete_solution(nx, ny, alpha, U):
    """Exact steady solution of the discrete equations (module docstring),
    [ny, nx]: column i at x = i + 1 from the inlet ghost, row j at y = j + 1
    from the lower wall.  Assumes the outlet far enough downstream that the
    growing root does not enter (r_n^nx negligible)."""
    L = ny + 1
    j = np.arange(1, ny + 1)
    out = np.zeros((ny, nx))
    i = np.arange(nx) + 1
    for n in range(1, ny + 1):
        s = np.sin(n * math.pi * j / L)
        b = 2.0 / L * np.sum(s)  # discrete sine coefficient of the uniform inflow
        if abs(b) < 1e-15:
            continue
        kap = 2.0 - 2.0 * math.cos(n * math.pi / L)
        a, bq, c = alpha, -(2.0 * alpha + alpha * kap + U), alpha + U
        disc = math.sqrt(bq * bq - 4.0 * a * c)
        r = (-bq - disc) / (2.0 * a)  # the root below one
        out += b * s[:, None] * r ** i[None, :]
    return out


def setup(ny, Pe=20.0, length_over_L=4.0, T_in=W.T_IN, dT=1e-4, precision="fp64"):
    """The plug-flow channel: L = ny + 1 and Pe = U L / alpha with
    alpha = min(0.08, 0.05 L / Pe) (nu = alpha Pr), U = alpha Pe / L: at
    most 0.05 (low Mach), and alpha within the explicit-stability bound;
    T_w = T_in + dT (a small difference keeps the density, and with it the
    flow, uniform to about dT/T)."""
    L = ny + 1
    alpha = min(0.08, 0.05 * L / Pe)
    U = alpha * Pe / L
    nx = int(round(length_over_L * L))
    s = W.base_setup(2, nx, ny, 1, 0, precision)
    s["lb_bc"] = ["inlet", "char_outlet", "periodic", "periodic", "periodic", "periodic"]
    s["outlet_sigma"] = 0.25
    T_w = T_in + dT
    s["fd_bc"] = ["dirichlet", "neumann", "dirichlet", "dirichlet", "periodic", "periodic"]
    s["fd_val"][0] = [T_in]
    s["fd_val"][2] = [T_w]
    s["fd_val"][3] = [T_w]
    s["T_in"] = T_in
    s["T_s"] = T_w
    s["A_T"] = 0.0
    s["mu_model"] = 0
    s["nu_in"] = alpha * s["Pr"]
    s["u_in"] = [U, 0.0, 0.0]
    return s, alpha


def run(ny, steps=None, tol=1e-11, **kw):
    """Steady GPU solution T^ on the [ny, nx] grid (and the setup, alpha)."""
    from . import lbfd

    s, alpha = setup(ny, **kw)
    shape = (1, ny, s["nx"])
    ctx = lbfd.Context(s, np.zeros(shape))
    u0 = np.zeros((2,) + shape)
    u0[0] = s["u_in"][0]
    ctx.init_state(np.full(shape, s["T_in"]), None, u0)
    dT = s["fd_val"][2][0] - s["T_in"]
    prev, done = None, 0
    chunk = 2000
    limit = steps or 2000000
    while done < limit:
        ctx.step(chunk)
        done += chunk
        That = (s["fd_val"][2][0] - ctx.fields()["T"][0]) / dT
        if prev is not None and np.abs(That - prev).max() < tol:
            break
        prev = That
    return That, s, alpha, done


def section_mse(That, s, alpha, x_over_L=1.0, axial=False):
    """Eq. mean-standard-error-f with f = T^ across the section x = x_over_L L
    against the series (axial: the one with axial conduction), over the
    whole width (no interface: eta = 0); the wall values (T^ = 0) close the
    profile."""
    from .calibration import mse

    ny = s["ny"]
    L = ny + 1
    i = int(round(x_over_L * L)) - 1
    y = np.concatenate([[0.0], np.arange(1, ny + 1), [L]])
    f_fd = np.concatenate([[0.0], That[:, i], [0.0]])
    ref = series_axial if axial else series
    f_ref = ref(i + 1, y, L, alpha, s["u_in"][0])
    return mse(f_ref, f_fd, y, L, 0.0)


def convergence(sizes=(8, 16, 32, 64, 128), Pe=20.0, log=None):
    rows = []
    for ny in sizes:
        That, s, alpha, n = run(ny, Pe=Pe)
        disc = discrete_solution(s["nx"], ny, alpha, s["u_in"][0])
        # the discrete solution away from the outlet: its zero-gradient ghost
        # adds a mode that decays upstream only by about (1 + U/alpha) per
        # column, so the last L columns are left out
        L = ny + 1
        dev = float(np.abs(That[:, :-L] - disc[:, :-L]).max())
        row = {"ny": ny, "L": L, "U": s["u_in"][0], "alpha": alpha, "steps": n,
               "max_dev_discrete": dev}
        for key, xl, ax in (("mse_x_L", 1.0, False), ("mse_x_2L", 2.0, False),
                            ("mse_axial_x_L", 1.0, True), ("mse_axial_x_2L", 2.0, True)):
            row[key] = section_mse(That, s, alpha, xl, ax)
        rows.append(row)
        if log:
            log(f"L = {L}: MSE vs series (x = L, 2L) {row['mse_x_L']:.3e} "
                f"{row['mse_x_2L']:.3e}; with axial conduction {row['mse_axial_x_L']:.3e} "
                f"{row['mse_axial_x_2L']:.3e}; |FD - discrete solution| {dev:.2e} ({n} steps)")
    for a, b in zip(rows, rows[1:]):
        for key in ("mse_x_L", "mse_x_2L", "mse_axial_x_L", "mse_axial_x_2L"):
            b["rate_" + key[4:]] = math.log(a[key] / b[key]) / math.log(b["L"] / a["L"])
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description="plug-flow Graetz convergence study")
    ap.add_argument("--Pe", type=float, default=20.0)
    ap.add_argument("--sizes", type=int, nargs="*", default=[8, 16, 32, 64, 128])
    ap.add_argument("--max-steps", type=int, default=2000000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    rows = convergence(a.sizes, a.Pe, log=lambda m: print(m, flush=True))
    res = {"command": "python -m paper_2310_17214_amd.graetz " + " ".join(argv or sys.argv[1:]),
           "Pe": a.Pe, "rows": rows}
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(json.dumps(res, indent=1) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
