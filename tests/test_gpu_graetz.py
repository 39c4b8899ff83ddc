"""Plug flow between isothermal walls on the GPU (FD Dirichlet temperatures
on LB-periodic faces): the steady state against the FP64 oracle and against
the exact solution of the discrete equations (Sec. 4.3 setting)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2310_17214_amd import graetz as G

pytestmark = pytest.mark.gpu


def test_plug_flow_thermal_entrance_fp64():
    from paper_2310_17214_amd import lbfd

    ny = 7
    s, alpha = G.setup(ny, Pe=20.0)
    shape = (1, ny, s["nx"])
    u0 = np.zeros((2,) + shape)
    u0[0] = s["u_in"][0]
    T0 = np.full(shape, s["T_in"])
    ctx = lbfd.Context(s, np.zeros(shape))
    ctx.init_state(T0, None, u0)
    ctx.step(20000)
    o = O.Oracle(s, np.zeros(shape))
    o.init_state(T0, None, u0)
    o.step(20000)
    T_w = s["fd_val"][2][0]
    dT = T_w - s["T_in"]
    th_g = (T_w - ctx.fields()["T"][0]) / dT
    th_o = (T_w - o.read(O.F_T)[0]) / dT
    print("max |gpu - oracle| in T^:", np.abs(th_g - th_o).max(), flush=True)
    assert np.abs(th_g - th_o).max() <= 1e-8  # 1e-12 of T, in units of dT = 1e-4 K
    disc = G.discrete_solution(s["nx"], ny, alpha, s["u_in"][0])
    assert np.abs(th_g[:, :-10] - disc[:, :-10]).max() <= 2e-7
    g, r = ctx.fields(), o.fields()
    for c in range(2):
        assert np.abs(g["u"][c] - r["u"][c]).max() <= 1e-12 * s["u_in"][0]
