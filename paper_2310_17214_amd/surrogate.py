"""Chemistry surrogate workflow on one GPU: sample training pairs from exact
runs, train, evaluate, install.  Orchestration of library calls only -- the
sampling, training and inference arithmetic runs in the HIP kernels.

Training pairs (x, y) are states of an exact run and the exact
step-integrated sources of one further step from them (one step of n_sub
FP64 sub-steps); cells are drawn uniformly by a seeded host generator every
`every` steps, and the draws are passed to the device as cell indices.
"""
from __future__ import annotations

import numpy as np

from . import lbfd

HIDDEN = lbfd.HIDDEN


def initial_weights(ns, seed):
    """He-uniform weights, zero biases, the output layer scaled by 0.1 (flat
    FP32 in the library's layout: W1, b1, W2, b2, W3, b3)."""
    rng = np.random.default_rng(seed)
    ni = 2 + ns

    def u(fan_in, shape, scale=1.0):
        b = np.sqrt(6.0 / fan_in)
        return (scale * rng.uniform(-b, b, shape)).astype(np.float32).ravel()

    parts = [u(ni, (HIDDEN, ni)), np.zeros(HIDDEN, np.float32), u(HIDDEN, (HIDDEN, HIDDEN)),
             np.zeros(HIDDEN, np.float32), u(HIDDEN, (ns, HIDDEN), 0.1), np.zeros(ns, np.float32)]
    return np.concatenate(parts)


def sample_run(wl, steps, every, per_snapshot, seed, ctx=None):
    """Exact run of `steps` steps from the workload's initial state, sampling
    `per_snapshot` cells at steps 0, every, 2 every, ..., steps.  Returns
    torch CUDA tensors x [n, 2 + ns], y [n, ns]."""
    import torch

    if ctx is None:
        ctx = lbfd.Context(wl.setup, wl.phi)
    ctx.init_state(wl.T0, wl.Y0)
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    done = 0
    while True:
        cells = torch.tensor(rng.integers(0, ctx.N, per_snapshot).astype(np.int32), device="cuda")
        x, y = ctx.sample_states(cells)
        xs.append(x)
        ys.append(y)
        if done >= steps:
            break
        n = min(every, steps - done)
        ctx.step(n)
        done += n
    ctx.synchronize()
    return torch.cat(xs), torch.cat(ys)


def split(x, y, holdout, seed):
    """Seeded random split into training and held-out pairs."""
    import torch

    n = x.shape[0]
    perm = torch.tensor(np.random.default_rng(seed).permutation(n), device=x.device)
    k = int(round(n * (1.0 - holdout)))
    tr, ho = perm[:k], perm[k:]
    return (x[tr].contiguous(), y[tr].contiguous()), (x[ho].contiguous(), y[ho].contiguous())


def train(x, y, ns, epochs=8, batch=4096, lr=2e-3, lr_final=2e-4, seed=4, log=None):
    """Adam on the training pairs; returns (weights, norm, envelope, losses)."""
    tr = lbfd.Trainer(ns, batch=batch)
    tr.fit_norm(x, y)
    tr.set_weights(initial_weights(ns, seed))
    losses = tr.fit(x, y, epochs=epochs, lr=lr, seed=seed + 1, lr_final=lr_final, log=log)
    w, norm, env = tr.export()
    return w, norm, env, losses


def heldout_rmse(ctx, x, y):
    """RMS error of the installed surrogate's raw prediction on held-out
    pairs, per species: (absolute [ns], relative to the targets' RMS [ns],
    share of fallback cells)."""
    ns = y.shape[1]
    raw, _, fb = ctx.surrogate_eval(x[:, 0].contiguous(), x[:, 2:].t().contiguous())
    d = (raw.t() - y).double()
    rmse = d.pow(2).mean(0).sqrt().cpu().numpy()
    ref = y.double().pow(2).mean(0).sqrt().cpu().numpy()
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(ref > 0, rmse / ref, np.nan)  # NaN: a species with no source (inert)
    return rmse, rel, float((fb != 0).float().mean().cpu())
