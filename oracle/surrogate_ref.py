"""CPU reference of the chemistry surrogate -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU baseline may import
this module.  It shares no code with the HIP kernels.

What the surrogate computes (a reading of the reaction step of the paper's
Lie split, Eqs. 8 and 9, replaced by a learned map; see the design notes):
the step-integrated chemical source of one time step,
    omega_bar_k = rho (Y_k^chem - Y_k) / dt,
where Y^chem is the exact n_sub-sub-step explicit Euler integration of the
Arrhenius sources from (T, Y) (the oracle's reactor), and the map
    x = (T, p, Y_1..Y_ns)  ->  omega_bar_1..omega_bar_ns
is a 2-hidden-layer ReLU perceptron of width 256.  In use its prediction is
de-standardised, checked (envelope, overdraw, residual, positivity), projected so that
the mass fractions keep their sum, and applied as one explicit update:
    Y_k += dt w_k / rho,  T += dt w_T / (rho c_p),  w_T = -sum_k dh_k w_k.

Functions:
  bf16_round            round-to-nearest-even to bfloat16 (values kept in float64)
  forward               the perceptron, optionally with the kernel's rounding points
  source                x -> (omega_hat, fallback flags) with all checks
  step_source           the exact target omega_bar from the oracle's reactor
  loss_and_grad         FP64 mean-square loss and its gradient (backpropagation)
  adam                  one Adam update (Kingma and Ba, 2015)
  fit_norm              standardisation statistics and the input envelope
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

HIDDEN = 256
RESID_TOL = 0.05
POS_TOL = -1e-8
CLIP_TOL = 0.05
ENV_MARGIN = 0.01      # of the envelope's range
ENV_MARGIN_SD = 0.05   # of the input's standard deviation
Y_SD_FLOOR = 1e-4      # mass-fraction inputs


def n_in(ns):
    return 2 + ns


def bf16_round(x):
    """float -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def init_weights(ns, seed, hidden=HIDDEN):
    """He-uniform initial weights, zero biases (float32 arrays)."""
    rng = np.random.default_rng(seed)
    ni, no = n_in(ns), ns
    def u(fan_in, shape):
        b = np.sqrt(6.0 / fan_in)
        return rng.uniform(-b, b, shape).astype(np.float32)
    return {"W1": u(ni, (hidden, ni)), "b1": np.zeros(hidden, np.float32),
            "W2": u(hidden, (hidden, hidden)), "b2": np.zeros(hidden, np.float32),
            "W3": u(hidden, (no, hidden)) * np.float32(0.1), "b3": np.zeros(no, np.float32)}


def pack(w):
    """Flat FP32 layout of the weights: W1, b1, W2, b2, W3, b3 (row-major)."""
    return np.concatenate([np.asarray(w[k], np.float32).ravel()
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unpack(flat, ns, hidden=HIDDEN):
    ni, no = n_in(ns), ns
    shapes = [("W1", (hidden, ni)), ("b1", (hidden,)), ("W2", (hidden, hidden)),
              ("b2", (hidden,)), ("W3", (no, hidden)), ("b3", (no,))]
    out, o = {}, 0
    for k, sh in shapes:
        n = int(np.prod(sh))
        out[k] = np.asarray(flat[o:o + n], np.float32).reshape(sh)
        o += n
    assert o == len(flat)
    return out


def sigma_floor(mu, sd):
    """Standard deviations floored at 1e-12 max(|mu|, 1) (constant inputs)."""
    return np.maximum(sd, 1e-12 * np.maximum(np.abs(mu), 1.0))


def fit_norm(X, Yt):
    """Mean and (floored, population) standard deviation of inputs and
    targets, and the per-feature input envelope [min, max].  The mass-fraction
    inputs (features 2..) have their standard deviation floored at
    Y_SD_FLOOR as well."""
    X, Yt = np.asarray(X, np.float64), np.asarray(Yt, np.float64)
    mx, my = X.mean(0), Yt.mean(0)
    sx = sigma_floor(mx, X.std(0))
    sx[2:] = np.maximum(sx[2:], Y_SD_FLOOR)
    sy = sigma_floor(my, Yt.std(0))
    return {"mu_x": mx, "sd_x": sx, "mu_y": my, "sd_y": sy, "lo": X.min(0), "hi": X.max(0)}


def forward(w, xhat, emulate=True):
    """Perceptron on standardised inputs xhat [n, n_in] -> yhat [n, n_out].

    emulate=True applies the kernel's rounding points: inputs, weights and
    both hidden activations rounded to bfloat16; products and sums exact
    (float64 here, float32 accumulation on the device); biases float32."""
    r = bf16_round if emulate else (lambda a: np.asarray(a, np.float64))
    W1, W2, W3 = r(w["W1"]), r(w["W2"]), r(w["W3"])
    b1, b2, b3 = (np.asarray(w[k], np.float64) for k in ("b1", "b2", "b3"))
    h1 = r(np.maximum(r(xhat) @ W1.T + b1, 0.0))
    h2 = r(np.maximum(h1 @ W2.T + b2, 0.0))
    return h2 @ W3.T + b3


def features(T, Y, p=1.0):
    T = np.atleast_1d(np.asarray(T, np.float64))
    Y = np.atleast_2d(np.asarray(Y, np.float64))
    return np.concatenate([T[:, None], np.full((len(T), 1), p), Y], axis=1)


def source(w, norm, setup, T, Y, p=1.0, emulate=True):
    """Surrogate source for cells with state (T, Y [n, ns]), dt = 1.

    Returns (omega [n, ns] after projection, omega_T [n], fallback [n] bool,
    raw [n, ns] de-standardised prediction after the overdraw clip, before
    the projection).  In order:
      overdraw: raw_k < -rho Y_k is clipped to -rho Y_k; an excess beyond
        CLIP_TOL sd_y[k] sends the cell to the exact path;
      residual: |sum raw| > RESID_TOL (sum |raw| + sum_k sd_y[k]) -> exact;
      projection: omega_k = raw_k - Y_k sum raw;
      positivity: Y_k + omega_k / rho < POS_TOL for some k -> exact;
      envelope: any input outside [lo - m, hi + m],
        m = ENV_MARGIN (hi - lo) + ENV_MARGIN_SD sd_x -> exact."""
    X = features(T, Y, p)
    Yv = X[:, 2:]
    xhat = (X - norm["mu_x"]) / norm["sd_x"]
    raw = norm["mu_y"] + norm["sd_y"] * forward(w, xhat, emulate)
    rho = np.array([O.eos(setup, t, y) for t, y in zip(X[:, 0], Yv)])
    floor = -rho[:, None] * Yv
    over = np.any(floor - raw > CLIP_TOL * norm["sd_y"], axis=1)
    raw = np.maximum(raw, floor)
    margin = (ENV_MARGIN * (np.asarray(norm["hi"]) - np.asarray(norm["lo"]))
              + ENV_MARGIN_SD * np.asarray(norm["sd_x"]))
    out_env = np.any((X < norm["lo"] - margin) | (X > norm["hi"] + margin), axis=1)
    resid = np.abs(raw.sum(1)) > RESID_TOL * (np.abs(raw).sum(1) + np.sum(norm["sd_y"]))
    omega = raw - Yv * raw.sum(1, keepdims=True)
    dhf = np.asarray(setup["mech"]["dhf"], np.float64)
    omega_T = -(omega * dhf).sum(1)
    neg = np.any(Yv + omega / rho[:, None] < POS_TOL, axis=1)
    return omega, omega_T, out_env | over | resid | neg, raw


def step_source(setup, T, Y):
    """Exact target: omega_bar = rho (Y_chem - Y)/dt over one step of n_sub
    explicit Euler sub-steps (the oracle's reactor), dt = 1."""
    T = np.atleast_1d(np.asarray(T, np.float64))
    Y = np.atleast_2d(np.asarray(Y, np.float64))
    out = np.empty_like(Y)
    for i in range(len(T)):
        rho = O.eos(setup, T[i], Y[i])
        _, Yc = O.reactor(setup, T[i], Y[i], 1)
        out[i] = rho * (np.asarray(Yc) - Y[i])
    return out


def loss_and_grad(w, xhat, yhat_target):
    """Mean-square loss L = mean over samples and outputs of (yhat - t)^2 of
    the un-rounded perceptron in float64, and dL/dw by backpropagation."""
    W1, W2, W3 = (np.asarray(w[k], np.float64) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (np.asarray(w[k], np.float64) for k in ("b1", "b2", "b3"))
    x = np.asarray(xhat, np.float64)
    t = np.asarray(yhat_target, np.float64)
    n, no = t.shape
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    L = float(np.mean((y - t) ** 2))
    d3 = 2.0 * (y - t) / (n * no)
    g = {"W3": d3.T @ h2, "b3": d3.sum(0)}
    d2 = (d3 @ W3) * (z2 > 0)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0)
    g["W1"], g["b1"] = d1.T @ x, d1.sum(0)
    return L, g


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t >= 1) in float64 on every array of w; returns the new
    (w, m, v)."""
    nw, nm, nv = {}, {}, {}
    for k in w:
        nm[k] = beta1 * m[k] + (1 - beta1) * g[k]
        nv[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = nm[k] / (1 - beta1 ** t)
        vh = nv[k] / (1 - beta2 ** t)
        nw[k] = w[k] - lr * mh / (np.sqrt(vh) + eps)
    return nw, nm, nv
