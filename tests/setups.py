"""Small seeded setups shared by the CPU and GPU tests (inputs only: no
method arithmetic)."""
import numpy as np

from paper_2310_17214_amd import workloads as W


def small_box(precision="fp64", ns=4):
    """3-D box with every boundary kind: inlet/outlet in x, walls in y,
    periodic z; ragged cell count (not a multiple of the workgroup)."""
    nx, ny, nz = 13, 10, 9
    s = W.base_setup(3, nx, ny, nz, ns, precision)
    s["lb_bc"] = ["inlet", "outlet", "wall", "wall", "periodic", "periodic"]
    s["fd_bc"] = ["dirichlet", "neumann", "neumann", "dirichlet", "periodic", "periodic"]
    s["mech"] = W.mech_one_step(A=W.one_step_rate_constant(tau_steps=5.0))
    s["Y_in"] = W.ONE_STEP_Y_IN
    s["fd_val"][0] = [300.0] + W.ONE_STEP_Y_IN
    s["fd_val"][3] = [900.0] + W.ONE_STEP_Y_BURNT
    s["u_in"] = [0.02, 0.0, 0.0]
    # within the explicit-stability rule up to 900 K (the library refuses
    # nu_in = 0.03 with T up to 1000 K: 2 d alpha alone is 1.9 there)
    s["nu_in"] = 0.008
    s["T_s"] = 800.0
    s["A_T"] = 90.0
    s["F_b"] = [0.0, 1e-5, 0.0]
    shape = (nz, ny, nx)
    phi = np.clip(0.5 + 0.6 * W.random_smooth_field(shape, 5), 0.0, 1.0)
    T0 = 700.0 + 200.0 * W.random_smooth_field(shape, 6)
    Y0 = np.stack([0.25 + 0.1 * W.random_smooth_field(shape, 10 + k) for k in range(4)])
    Y0 /= Y0.sum(0)
    u0 = np.stack([0.01 * W.random_smooth_field(shape, 20 + a) for a in range(3)])
    return s, phi, T0, Y0, u0
