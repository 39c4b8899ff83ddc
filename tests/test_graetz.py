"""Closed forms of the plug-flow thermal entrance (Sec. 4.3, Eq.
graetz_solution) used by the convergence study: the series, its variant with
axial conduction, and the exact solution of the discrete FD equations."""
import math

import numpy as np

from paper_2310_17214_amd import graetz as G


def test_series_is_the_inflow_at_the_inlet_and_zero_on_the_walls():
    L = 10.0
    y = np.array([0.0, 2.5, 5.0, 7.5, L])
    t0 = G.series(0.0, y, L, 0.1, 0.05, nterms=4000)
    assert abs(t0[0]) < 1e-12 and abs(t0[-1]) < 1e-12
    assert np.abs(t0[1:-1] - 1.0).max() < 1e-3  # the Fourier series of 1
    # one mode far downstream: 4/pi sin(pi y/L) exp(-(pi/L)^2 alpha x/U)
    x = 400.0
    ref = 4 / math.pi * np.sin(math.pi * y / L) * math.exp(-(math.pi / L) ** 2 * 0.1 * x / 0.05)
    assert np.abs(G.series(x, y, L, 0.1, 0.05) - ref).max() <= 1e-12


def test_axial_series_tends_to_the_series_at_large_peclet():
    y = np.linspace(0.0, 10.0, 11)
    for x, alpha in ((1.0, 1e-6), (5.0, 1e-4), (20.0, 1e-4)):
        d = np.abs(G.series_axial(x, y, 10.0, alpha, 1.0) - G.series(x, y, 10.0, alpha, 1.0))
        assert d.max() < 1e-9
    # at a moderate Peclet number axial conduction slows the decay
    assert G.series_axial(30.0, 5.0, 10.0, 0.2, 0.1) > G.series(30.0, 5.0, 10.0, 0.2, 0.1)


def test_discrete_solution_solves_the_discrete_equations():
    """Residual of the steady upwind/central equations with the ghosts
    (walls 0, inlet 1) at every interior column: round-off."""
    ny, nx, alpha, U = 9, 60, 0.03, 0.05
    T = G.discrete_solution(nx, ny, alpha, U)
    P = np.zeros((ny + 2, nx + 1))
    P[1:-1, 1:] = T
    P[1:-1, 0] = 1.0  # inlet ghost
    c = P[1:-1, 1:-1]
    adv = U * (c - P[1:-1, :-2])
    lap = (P[1:-1, 2:] - 2 * c + P[1:-1, :-2]) + (P[2:, 1:-1] - 2 * c + P[:-2, 1:-1])
    res = adv - alpha * lap
    assert np.abs(res).max() <= 1e-15
    assert np.abs(T[:, 0] - 1.0).max() < 0.5 and T[:, -1].max() < 0.2
