"""Checks of the seeded input generators (data only, no method arithmetic)."""
import itertools
import math

import numpy as np

from paper_2310_17214_amd import workloads as W


def test_synthetic_mechanism_is_element_and_mass_balanced():
    m = W.mech_synthetic9()
    comp = np.array(W._SPECIES)
    s = np.array(m["nu_r"]) - np.array(m["nu_f"])
    assert s.shape == (21, 9)
    assert np.all(s @ comp == 0)                      # every pseudo-element balanced
    assert np.allclose(s @ np.array(m["M"]), 0.0)     # hence mass balanced
    assert np.all(s[:, 8] == 0)                       # the diluent never reacts
    assert all(m["rev"]) and 1 <= m["n_sub"] <= 32
    # initiation from the fresh mixture exists
    nu_f = np.array(m["nu_f"])
    assert any(nu_f[j, 0] == 1 and nu_f[j, 1] == 1 for j in range(21))


def test_synthetic_equilibrium_constants_are_cycle_consistent():
    """ln Kc_j(T) = sum_k s_kj g_k(T) must have an exact solution g (species
    potentials) at every T: then every reaction cycle has prod Kc = 1."""
    m = W.mech_synthetic9()
    s = np.array(m["nu_r"]) - np.array(m["nu_f"])
    for T in (600.0, 1500.0):
        lnK = np.array(m["lnKc_a"]) + np.array(m["lnKc_b"]) / T
        g, *_ = np.linalg.lstsq(s, lnK, rcond=None)
        assert np.abs(s @ g - lnK).max() < 1e-9 * max(1.0, np.abs(lnK).max())


def test_burnt_composition_conserves_elements():
    comp = np.array(W._SPECIES, float)
    M = comp @ W._ELEM_MASS
    e_in = (np.array(W.SYNTH9_Y_IN) / M) @ comp
    e_b = (np.array(W.burnt_synth9()) / M) @ comp
    assert np.allclose(e_in, e_b) and abs(sum(W.burnt_synth9()) - 1) < 1e-12
    # one-step mechanism: lean, all fuel burnt
    assert abs(sum(W.ONE_STEP_Y_IN) - 1) < 1e-15 and abs(sum(W.ONE_STEP_Y_BURNT) - 1) < 1e-15
    assert W.ONE_STEP_Y_IN[0] < W.ONE_STEP_Y_IN[1]


def test_one_step_rate_constant_sets_the_time_scale():
    A = W.one_step_rate_constant()
    assert abs(1.0 / (A * math.exp(-15000.0 / 1100.0) * (300.0 / 1100.0) * 0.5) - 50.0) < 1e-9


def test_sphere_packing_has_no_overlaps_and_target_porosity():
    shape = (48, 48, 96)
    parts = W.sphere_bed(shape, (16, 80), 8.0, 0.40, seed=7)
    c = np.array([p.centre for p in parts])
    for i, j in itertools.combinations(range(len(c)), 2):
        d = c[i] - c[j]
        d[1:] -= 48 * np.round(d[1:] / 48)  # periodic y, z
        assert np.linalg.norm(d) >= 16.0 - 1e-6
    por = W.bed_porosity(W.sharp_solid(shape, parts, (False, True, True)), (16, 80))
    assert abs(por - 0.40) < 0.03


def test_phase_profiles():
    d = np.linspace(-6, 6, 121)
    t = W.phase_tanh(d, 4.0)
    s = W.phase_sine(d, 4.0)
    assert np.all(np.diff(t) < 0) and np.all((t > 0) & (t < 1))
    assert t[60] == 0.5 and s[60] == 0.5  # interface at d = 0
    # same slope at the centre, -pi/(2 eta)
    slope_t = (t[61] - t[59]) / (d[61] - d[59])
    slope_s = (s[61] - s[59]) / (d[61] - d[59])
    assert abs(slope_t + math.pi / 8) < 1e-3 and abs(slope_s + math.pi / 8) < 1e-3
    assert s[0] == 1.0 and s[-1] == 0.0


def test_cfg1_parameters():
    wl = W.cylinder_channel()
    s = wl.setup
    assert (s["nx"], s["ny"]) == (128, 64) and wl.steps == 2000
    assert abs(s["u_in"][0] * 20.0 / s["nu_in"] - 20.0) < 1e-12   # Re = 20 on D = 20
    assert abs(s["T_s"] - 450.0) < 1e-12
    assert wl.phi[0, 32, 32] > 0.99 and wl.phi[0, 5, 100] < 1e-6


def test_slab_window_is_a_slice_of_the_whole_bed():
    """A window of the elongated bed (one GPU's share in a slab decomposition)
    holds exactly the phase field, temperature and composition of those
    cells of the whole bed."""
    kw = dict(nx=96, ny=16, nz=16, bed=(8, 88), x_split=40, steps=0)
    full = W.bed_elongated_9sp(**kw)
    part = W.bed_elongated_9sp(window=(30, 58), **kw)
    assert part.phi.shape == (16, 16, 28) and part.setup["nx"] == 28
    assert np.array_equal(part.phi, full.phi[:, :, 30:58])
    assert np.array_equal(part.T0, full.T0[:, :, 30:58])
    assert np.array_equal(part.Y0, full.Y0[:, :, :, 30:58])
    kinds = {p.kind for p in full.particles}
    assert kinds == {"sphere", "superquadric"}
    solid = W.sharp_solid(full.phi.shape, full.particles, (False, True, True))
    assert abs(W.bed_porosity(solid, full.bed) - 0.40) < 0.06
