"""Species heat capacities c_p,k on the GPU (HIP, gfx950) against the FP64
oracle, through the C ABI: the mixture c_p per cell and the species
heat-flux term of the temperature equation.  Bars as elsewhere: FP64 mode
<= 1e-12 per field, FP32 mode after 1000 steps u <= 1e-5, T and Y_k <=
1e-4."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2310_17214_amd import workloads as W

pytestmark = pytest.mark.gpu


def lb():
    from paper_2310_17214_amd import lbfd

    return lbfd


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def say(*a):
    print(*a, flush=True)


def _errs(ctx, orc):
    g, r = ctx.fields(), orc.fields()
    errs = {k: rel(g[k], r[k]) for k in ("T", "Ph", "rho", "divu")}
    for c in range(r["u"].shape[0]):
        errs[f"u{c}"] = rel(g["u"][c], r["u"][c])
    for c in range(r["Y"].shape[0]):
        errs[f"Y{c}"] = rel(g["Y"][c], r["Y"][c])
    return errs


def _with_cp(wl, factors):
    wl.setup["mech"] = dict(wl.setup["mech"], cp=[wl.setup["cp"] * f for f in factors])
    return wl


def _crop(precision, theta=0.01):
    wl = W.bed_one_step(nx=129, ny=17, nz=15, precision=precision, bed=(8, 121), x_split=60,
                        steps=0)
    wl.setup["theta_ign"] = theta
    return _with_cp(wl, [1.0, 1.3, 0.8, 1.1])


def _run(wl, steps):
    ctx = lb().Context(wl.setup, wl.phi)
    ctx.init_state(wl.T0, wl.Y0)
    ctx.step(steps)
    o = O.Oracle(dict(wl.setup, precision="fp64"), wl.phi)
    o.init_state(wl.T0, wl.Y0)
    o.step(steps)
    return ctx, o


def test_exponential_profile_of_the_species_heat_flux_fp64():
    """The oracle pin's setting (three inert species, uniform mixture c_p,
    linear mass fractions) on the GPU: the steady temperature is the exact
    discrete exponential profile, and the GPU equals the oracle."""
    nx = 10
    s = W.base_setup(2, nx, 1, 1, 3)
    s["lb_bc"] = ["wall", "wall", "periodic", "periodic", "periodic", "periodic"]
    s["fd_bc"] = ["dirichlet", "dirichlet", "periodic", "periodic", "periodic", "periodic"]
    YL, YR, TL, TR = [0.2, 0.5, 0.3], [0.4, 0.1, 0.5], 300.0, 420.0
    s["fd_val"][0] = [TL] + YL
    s["fd_val"][1] = [TR] + YR
    s["mu_model"], s["nu_in"] = 0, 0.03  # within the stability rule (D = 2 alpha)
    s["Le"] = [1.0, 2.0 / 3.0, 0.5]
    s["Y_in"] = YL
    cp0 = s["cp"]
    s["mech"] = dict(W.mech_empty(3), cp=[cp0, 1.5 * cp0, 2.0 * cp0])
    shape = (1, 1, nx)
    Y0 = np.stack([np.full(shape, 0.3), np.full(shape, 0.3), np.full(shape, 0.4)])
    T0 = np.full(shape, 350.0)
    ctx = lb().Context(s, np.zeros(shape))
    ctx.init_state(T0, Y0)
    ctx.step(60000)
    o = O.Oracle(s, np.zeros(shape))
    o.init_state(T0, Y0)
    o.step(60000)
    T = ctx.fields()["T"][0, 0]
    assert rel(T, o.read(O.F_T)[0, 0]) <= 1e-12
    x = np.arange(nx)
    mu = s["rho_in"] * s["nu_in"]
    lam = mu * cp0 * 1.55 / s["Pr"]
    g = np.array(YR) - np.array(YL)
    B = float(np.sum(cp0 * np.array([1.0, 1.5, 2.0]) * mu / (s["Pr"] * np.array(s["Le"])) * g))
    B /= nx + 1
    r = (lam - B / 2) / (lam + B / 2)
    C = (TR - TL) / (r ** (nx + 1) - 1.0)
    assert np.abs(T - (TL - C + C * r ** (x + 1))).max() <= 1e-10 * TR


def test_bed_crop_with_species_heat_capacities_fp64():
    wl = _crop("fp64")
    say("one-step crop with c_p,k, fp64 300 steps")
    ctx, o = _run(wl, 300)
    errs = _errs(ctx, o)
    say(errs)
    assert max(errs.values()) <= 1e-12, errs
    dg, do = ctx.diagnostics(), o.diag()
    assert abs(dg["enthalpy"] - do[O.D_ENTHALPY]) <= 1e-12 * abs(do[O.D_ENTHALPY])
    assert dg["n_flagged_fp64"] == do[O.D_FLAGGED] > 0


@pytest.mark.parametrize("theta", [0.01, 1.0])
def test_bed_crop_with_species_heat_capacities_fp32_1000_steps(theta):
    wl32, wl64 = _crop("fp32", theta), _crop("fp64", theta)
    say(f"one-step crop with c_p,k, fp32 1000 steps, theta {theta} K")
    ctx = lb().Context(wl32.setup, wl32.phi)
    ctx.init_state(wl32.T0, wl32.Y0)
    ctx.step(1000)
    o = O.Oracle(wl64.setup, wl64.phi)
    o.init_state(wl64.T0, wl64.Y0)
    o.step(1000)
    errs = _errs(ctx, o)
    say(errs)
    for k, e in errs.items():
        if k.startswith("u"):
            assert e <= 1e-5, (k, e)
        if k == "T" or k.startswith("Y"):
            assert e <= 1e-4, (k, e)


def test_nine_species_crop_with_species_heat_capacities_fp64():
    wl = W.bed_sphere_9sp(nx=129, ny=18, nz=14, precision="fp64", bed=(8, 121), x_split=60,
                          steps=0, T_burnt=1400.0)
    wl.setup["nu_in"] = 0.004
    wl.setup["theta_ign"] = 0.01
    _with_cp(wl, [1.0, 0.9, 1.2, 1.1, 0.95, 1.05, 1.3, 0.85, 1.0])
    say("nine-species crop with c_p,k, fp64 100 steps")
    ctx, o = _run(wl, 100)
    errs = _errs(ctx, o)
    say(errs)
    assert max(errs.values()) <= 1e-12, errs


def test_species_heat_capacity_arguments_are_checked():
    wl = _crop("fp64")
    s = wl.setup
    for bad in (dict(transport=1), dict(chem_scheme=1), dict(si=1)):
        with pytest.raises(Exception):
            lb().Context(dict(s, **bad), wl.phi)
    with pytest.raises(Exception):
        lb().Context(dict(s, mech=dict(s["mech"], cp=[1.0, -1.0, 1.0, 1.0])), wl.phi)
