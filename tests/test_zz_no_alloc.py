"""The entry point that allocates nothing (lbfd_fit_norm_noalloc) against the
trainer path it stands in for (lbfd_trainer_fit_norm + lbfd_trainer_export),
through the C ABI, on two calls in a row -- the second with fewer samples and
fewer species, so that the shared device staging block must not carry
anything over -- and the argument checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def lb():
    from paper_2310_17214_amd import lbfd

    return lbfd


def _pairs(n, ns, seed):
    import torch

    rng = np.random.default_rng(seed)
    T = rng.uniform(300.0, 1800.0, n)
    Y = rng.dirichlet(np.full(ns, 0.6), size=n)
    x = np.concatenate([T[:, None], np.ones((n, 1)), Y], axis=1).astype(np.float32)
    y = (rng.standard_normal((n, ns)) * np.logspace(-6, -2, ns)).astype(np.float32)
    return torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")


def _trainer_norm(ns, x, y):
    tr = lb().Trainer(ns, batch=256)
    tr.fit_norm(x, y)
    tr.set_weights(np.zeros(tr.np, np.float32))
    _, nrm, env = tr.export()
    return nrm, env


def test_noalloc_statistics_equal_the_trainer_path_on_two_calls():
    L = lb()
    for n, ns, seed in ((200_003, 9, 1), (5_001, 4, 2)):
        print(f"fit_norm_noalloc: n={n} ns={ns}", flush=True)
        x, y = _pairs(n, ns, seed)
        nrm, env = L.fit_norm_noalloc(ns, x, y)
        ref_n, ref_e = _trainer_norm(ns, x, y)
        assert nrm.shape == ref_n.shape and env.shape == ref_e.shape
        # same kernel, same order of every sum: bitwise equal
        assert np.array_equal(nrm, ref_n), np.abs(nrm - ref_n).max()
        assert np.array_equal(env, ref_e)
        # and the statistics are those of the data
        xh = x.double().cpu().numpy()
        np.testing.assert_allclose(nrm[: ns + 2], xh.mean(0), rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(env[: ns + 2], xh.min(0), rtol=0, atol=0)


def test_noalloc_argument_checks():
    import ctypes as C

    import torch

    L = lb()
    x, y = _pairs(64, 4, 3)
    fp = C.POINTER(C.c_float)
    out = np.empty(64, np.float32)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    f = L.lib().lbfd_fit_norm_noalloc
    assert f(15, x.data_ptr(), y.data_ptr(), 64, out.ctypes.data_as(fp), None, s) == \
        L.LBFD_E_UNSUPPORTED
    assert f(0, x.data_ptr(), y.data_ptr(), 64, out.ctypes.data_as(fp), None, s) == \
        L.LBFD_E_UNSUPPORTED
    assert f(4, x.data_ptr(), y.data_ptr(), 1, out.ctypes.data_as(fp), None, s) == L.LBFD_E_INVAL
    assert f(4, None, y.data_ptr(), 64, out.ctypes.data_as(fp), None, s) == L.LBFD_E_INVAL
    assert f(4, x.data_ptr(), y.data_ptr(), 64, None, None, s) == L.LBFD_E_INVAL
