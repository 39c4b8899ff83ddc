"""Surrogate training on the GPU against the CPU reference (S2 on the device).

The device gradient uses bf16 operands (activations, deltas, weights) with
FP32 accumulation, so it is compared with the FP64 reference gradient at the
bf16 level; the Adam update is compared with the formula given the same
gradient; standardisation statistics with numpy.
"""
import numpy as np
import pytest

from oracle import surrogate_ref as S

pytestmark = pytest.mark.gpu


def lb():
    from paper_2310_17214_amd import lbfd

    return lbfd


def say(*a):
    print(*a, flush=True)


NS = 9


def _data(n, seed):
    """States shaped like the bed's (T, p, Y) and a smooth target map."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(300.0, 2000.0, n)
    Y = rng.dirichlet(np.full(NS, 0.7), size=n)
    X = S.features(T, Y).astype(np.float32)
    t = (T - 1000.0) / 500.0
    Yt = np.stack([np.sin(1.3 * t + k) * Y[:, k] + 0.3 * Y[:, (k + 1) % NS] * t
                   for k in range(NS)], axis=1) * 1e-3
    return X, Yt.astype(np.float32)


def _start(seed):
    w = S.init_weights(NS, seed)
    rng = np.random.default_rng(seed + 100)
    w["b1"] = (0.05 * rng.normal(size=256)).astype(np.float32)
    w["b2"] = (0.05 * rng.normal(size=256)).astype(np.float32)
    return w


def _trainer(batch, X, Yt):
    import torch

    tr = lb().Trainer(NS, batch=batch)
    x = torch.tensor(X, device="cuda")
    y = torch.tensor(Yt, device="cuda")
    tr.fit_norm(x, y)
    return tr, x, y


def test_norm_statistics_match_numpy():
    X, Yt = _data(5000, 1)
    tr, x, y = _trainer(256, X, Yt)
    tr.set_weights(S.pack(_start(0)))
    _, nrm, env = tr.export()
    ref = S.fit_norm(X.astype(np.float64), Yt.astype(np.float64))
    ni = NS + 2
    got = {"mu_x": nrm[:ni], "sd_x": nrm[ni:2 * ni], "mu_y": nrm[2 * ni:2 * ni + NS],
           "sd_y": nrm[2 * ni + NS:], "lo": env[:ni], "hi": env[ni:]}
    for k in got:
        assert np.allclose(got[k], ref[k], rtol=1e-6, atol=1e-30), k
    assert got["sd_x"][1] == pytest.approx(1e-12)  # constant pressure input


def test_gradient_matches_the_reference_at_bf16_level():
    import torch

    B = 1024
    X, Yt = _data(3000, 2)
    tr, x, y = _trainer(B, X, Yt)
    w = _start(3)
    tr.set_weights(S.pack(w))
    idx = np.random.default_rng(4).choice(3000, B, replace=False).astype(np.int32)
    say("trainer gradient, batch 1024")
    g, loss = tr.gradient(x, y, torch.tensor(idx, device="cuda"))
    _, nrm, _ = tr.export()
    ni = NS + 2
    mu_x, sd_x = nrm[:ni].astype(np.float64), nrm[ni:2 * ni].astype(np.float64)
    mu_y, sd_y = nrm[2 * ni:2 * ni + NS].astype(np.float64), nrm[2 * ni + NS:].astype(np.float64)
    xh = (X[idx].astype(np.float64) - mu_x) / sd_x
    th = (Yt[idx].astype(np.float64) - mu_y) / sd_y
    L, gr = S.loss_and_grad(w, xh, th)
    say(f"loss device {loss:.6e} reference {L:.6e}")
    assert loss == pytest.approx(L, rel=2e-2)
    gd = S.unpack(g, NS)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        a, b = gd[k].astype(np.float64).ravel(), gr[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        say(f"{k}: relative error {rel:.3e} cosine {cos:.6f}")
        assert rel <= 3e-2 and cos >= 0.999, k


def test_adam_step_matches_the_formula():
    import torch

    B = 512
    X, Yt = _data(2048, 5)
    tr, x, y = _trainer(B, X, Yt)
    w0 = _start(6)
    tr.set_weights(S.pack(w0))
    idx = torch.tensor(np.arange(B, dtype=np.int32), device="cuda")
    g, _ = tr.gradient(x, y, idx)
    tr.step(x, y, idx, 1e-3)
    w1, _, _ = tr.export()
    zero = {k: np.zeros(v.shape) for k, v in w0.items()}
    w0d = {k: v.astype(np.float64) for k, v in w0.items()}
    gd = {k: v.astype(np.float64) for k, v in S.unpack(g, NS).items()}
    ref, _, _ = S.adam(w0d, gd, zero, zero, 1, lr=1e-3)
    got = S.unpack(w1, NS)
    scale = max(np.abs(v).max() for v in w0d.values())
    for k in ref:
        err = np.abs(got[k] - ref[k]).max()
        assert err <= 1e-6 * scale, (k, err)


def test_training_reduces_the_loss_and_exports_to_the_inference_kernel():
    import torch

    from paper_2310_17214_amd import workloads as W

    X, Yt = _data(32768, 7)
    tr, x, y = _trainer(1024, X, Yt)
    tr.set_weights(S.pack(_start(8)))
    say("training 6 epochs of 32 batches")
    hist = tr.fit(x, y, epochs=6, lr=2e-3, seed=9, lr_final=5e-4, log=say)
    assert hist[-1] < 0.1 * hist[0], hist
    w, nrm, env = tr.export()
    # the exported model in a context: inference against the reference
    wl = W.bed_superquadric_9sp(nx=12, ny=8, nz=8, precision="fp32", bed=(2, 10), x_split=6, steps=0)
    ctx = lb().Context(wl.setup, wl.phi)
    ctx.set_surrogate(w, nrm, env)
    n = 2000
    T = torch.tensor(X[:n, 0], device="cuda")
    Yd = torch.tensor(X[:n, 2:].T.copy(), device="cuda")
    raw, _, _ = ctx.surrogate_eval(T, Yd)
    raw = raw.cpu().numpy().T
    ni = NS + 2
    norm = {"mu_x": nrm[:ni].astype(np.float64), "sd_x": nrm[ni:2 * ni].astype(np.float64),
            "mu_y": nrm[2 * ni:2 * ni + NS].astype(np.float64),
            "sd_y": nrm[2 * ni + NS:].astype(np.float64),
            "lo": env[:ni].astype(np.float64), "hi": env[ni:].astype(np.float64)}
    _, _, _, ref_raw = S.source(S.unpack(w, NS), norm, wl.setup, X[:n, 0].astype(np.float64),
                                X[:n, 2:].astype(np.float64))
    err = np.abs(raw - ref_raw) / norm["sd_y"]
    say(f"exported model, standardised error median {np.median(err):.2e} max {err.max():.2e}")
    assert np.median(err) <= 1e-5 and np.mean(err > 1e-3) <= 1e-3
    # and it learned the map: error against the targets well below their spread
    fit = np.sqrt(np.mean(((raw - Yt[:n]) / norm["sd_y"]) ** 2))
    say(f"standardised RMS error against the targets {fit:.3e}")
    assert fit < 0.3
