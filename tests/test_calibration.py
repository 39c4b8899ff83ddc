"""Host-side pieces of the coupling-constant calibration (Sec. 4): the mean
standard error of Eq. mean-standard-error-f against hand-computed values and
a closed form, the minimum refinement, and the channel inputs."""
import math

import numpy as np
import pytest

from paper_2310_17214_amd import calibration as C


def test_mse_hand_computed_case():
    """L = 4, eta = 2, samples at the cell centres 0.5 .. 3.5:
    f_SI = (1, 2, 2, 1), f_DI = 1 -> d = (0, 1/2, 1/2, 0) after dividing by
    f_SI,max = 2.  Over [1, 3] the interpolant runs 1/4 -> 1/2 on [1, 1.5],
    stays 1/2 on [1.5, 2.5] and falls back to 1/4 on [2.5, 3]:
    int d^2 = 2 * (1/2)(1/16 + 1/8 + 1/4)/3 + 1/4 = 7/48 + 1/4 = 19/48, and
    MSE = (19/48) / (L - eta) = 19/96."""
    x = np.array([0.5, 1.5, 2.5, 3.5])
    e = C.mse([1, 2, 2, 1], [1, 1, 1, 1], x, 4.0, 2.0)
    assert e == pytest.approx(19.0 / 96.0, rel=1e-15)


def test_mse_linear_difference_closed_form():
    """f_SI = c and f_DI = c (1 + a (x - L/2)): the normalised difference is
    linear, and 1/(L - eta) int_{eta/2}^{L - eta/2} a^2 (x - L/2)^2 dx
    = a^2 (L - eta)^2 / 12, for any sampling that brackets the range."""
    L, eta, a, c = 50.0, 8.0, 3e-3, 0.07
    for n in (50, 137):
        x = np.linspace(0.25, L - 0.25, n)
        f_di = c * (1 + a * (x - L / 2))
        e = C.mse(np.full(n, c), f_di, x, L, eta)
        assert e == pytest.approx(a * a * (L - eta) ** 2 / 12.0, rel=1e-12)


def test_mse_invariances_and_range_checks():
    x = np.arange(50) + 0.5
    f = np.sin(x / 50 * np.pi)
    g = f + 0.01 * np.cos(x)
    assert C.mse(f, f, x, 50, 8) == 0.0
    assert C.mse(7 * f, 7 * g, x, 50, 8) == pytest.approx(C.mse(f, g, x, 50, 8), rel=1e-14)
    # only the bulk range [4, 46] counts: samples that do not bracket it
    # (3.5 and 46.5 do, through the interpolant) leave the error unchanged
    h = g.copy()
    h[x < 3] += 1.0
    h[x > 47] -= 1.0
    assert C.mse(f, h, x, 50, 8) == pytest.approx(C.mse(f, g, x, 50, 8), rel=1e-14)
    with pytest.raises(ValueError):
        C.mse(f, g, x, 50, 0.5)  # range starts before the first sample
    with pytest.raises(ValueError):
        C.mse(f, g, x, 50, 60)


def test_refine_minimum_of_a_parabola_in_log_a():
    vals = [20.0, 50.0, 100.0, 200.0, 400.0]
    xs = np.log(vals)
    x0 = math.log(137.0)
    errs = 1e-4 + 3e-5 * (xs - x0) ** 2
    best, bracketed = C.refine_minimum(vals, errs)
    assert bracketed and best == pytest.approx(137.0, rel=1e-10)
    best, bracketed = C.refine_minimum(vals, errs[::-1] * 0 + np.arange(5))
    assert not bracketed and best == 20.0


@pytest.mark.parametrize("eta", [4.0, 8.0])
def test_channel_geometry(eta):
    """The walls sit half-way between the last solid (phi >= 1/2) and the
    first fluid row: L fluid rows between eta/2 solid rows on each side; the
    profile is 1/2 at each wall and symmetric; the uniform inflow covers the
    fluid rows only, and Re = L u0 / nu."""
    L = 50
    s, phi, T0, prof, y = C.channel(L=L, eta=eta, si=True)
    row = phi[0, :, 0]
    assert s["ny"] == L + int(eta) and s["nx"] == 5 * L
    assert np.count_nonzero(row < 0.5) == L
    assert np.count_nonzero(row >= 0.5) == int(eta)
    assert np.allclose(row, row[::-1], rtol=0, atol=1e-15)
    assert C.wall_profile(np.array([0.0, L]), L, eta).tolist() == [0.5, 0.5]
    assert np.array_equal(prof[0, 0] > 0, row < 0.5)
    assert s["nu_in"] * 100.0 == pytest.approx(L * s["u_in"][0])
    st, _, T0t, pt, _ = C.channel(L=L, eta=eta, thermal=True)
    # fully developed inflow: a parabola over the fluid rows with mean ~u0
    fl = row < 0.5
    assert pt[0, 0, fl].mean() == pytest.approx(st["u_in"][0], rel=1e-3)
    assert st["fd_val"][2][0] == 400.0 and st["T_s"] == 400.0
