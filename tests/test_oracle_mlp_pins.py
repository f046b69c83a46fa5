"""Pins of the FP64 surrogate reference (CPU): explicit back-propagation
against central finite differences and against torch's FP64 autograd; the
bfloat16 rounding against known values; Adam training on a smooth target;
and the host-side data set construction of the library."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2110_14494_amd import workloads as W


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-2, 2, n)
    t = np.stack([np.sin(x * (k + 1) * 0.7) + 0.1 * k for k in range(6)], axis=1)
    mask = (rng.random((n, 6)) > 0.1).astype(np.float64)
    return x, t, mask


def test_parameter_count():
    assert M.N_PARAMS == 4678
    th = W.mlp_init(4)
    assert th.size == 4678 and np.allclose(M.pack(M.unpack(th)), th)


def test_gradient_matches_central_differences():
    x, t, mask = _data(50, 1)
    th = W.mlp_init(3) + np.random.default_rng(2).normal(0, 0.05, M.N_PARAMS)
    L, g = M.loss_and_grad(th, x, t, mask)
    h = 1e-6
    idx = np.random.default_rng(5).choice(M.N_PARAMS, 300, replace=False)
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss_only(th + e, x, t, mask) - M.loss_only(th - e, x, t, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    x, t, mask = _data(77, 2)
    th = W.mlp_init(6)
    L, g = M.loss_and_grad(th, x, t, mask)
    tt = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    p, o = {}, 0
    for name, shp in M.SHAPES:
        n = int(np.prod(shp))
        p[name] = tt[o:o + n].reshape(shp)
        o += n
    X = torch.tensor(x).reshape(-1, 1)
    h1 = torch.tanh(X @ p["W1"].T + p["b1"])
    h2 = torch.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    m = torch.tensor(mask)
    loss = ((y - torch.tensor(t)) ** 2 * m).sum() / m.sum()
    loss.backward()
    assert abs(loss.item() - L) < 1e-12 * max(1.0, L)
    np.testing.assert_allclose(tt.grad.numpy(), g, rtol=1e-10, atol=1e-14)


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -2.0 - 2 ** -7, 3.0e-3])
    r = M.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0  # a tie rounds to even
    assert r[2] == 1 + 2 ** -7
    assert r[3] == -2.0  # halfway between -2 and -2 - 2^-6: ties to the even mantissa
    assert abs(r[4] / 3.0e-3 - 1) < 2 ** -8


def test_adam_training_fits_smooth_targets():
    x, t, mask = _data(256, 7)
    th0 = W.mlp_init(4)
    th, losses = M.train(th0, x, t, mask, epochs=1500, lr0=3e-3, lr_min=1e-5)
    assert losses[-1] < 1e-2 * losses[0]
    # the cosine schedule ends at lr_min
    assert abs(M.cosine_lr(1500, 1500, 3e-3, 1e-5) - 1e-5) < 1e-18


def test_library_dataset_construction():
    # pcmcc_mlp_dataset is host code in the library (no device work).
    from paper_2110_14494_amd import surrogate as S
    from paper_2110_14494_amd import _binding as B
    n = 40
    EN = np.geomspace(10, 1000, n)
    rng = np.random.default_rng(3)
    vals = np.abs(rng.normal(1.0, 0.2, (n, B.SWARM_NQ))) + 0.1
    errs = 0.01 * vals
    vals[3, 11] = 0.0  # alpha = 0: masked
    errs[5, 12] = 0.5 * vals[5, 12]  # eta unresolved: masked
    vals[7, 2] = np.nan
    N = 2.45e25
    x, t, m, ln, sig, norm = S.dataset(EN, vals, errs, N, max_rel_err=0.1)
    q = {k: i for i, k in enumerate(B.SWARM_QUANTITIES)}
    ref = np.stack([vals[:, q["mu"]] * N, vals[:, q["DL_flux"]] * N, vals[:, q["alpha"]] / N,
                    vals[:, q["eta"]] / N, vals[:, q["mean_eps"]], vals[:, q["bulk_flux_ratio"]]], axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        lr = np.log(ref)
    ok = np.isfinite(lr)
    ok[5, 3] = False
    assert np.array_equal(m.astype(bool), ok)
    o = norm.opts
    assert abs(o.mu_x - np.log(EN).mean()) < 1e-12 and abs(o.sd_x - np.log(EN).std(ddof=1)) < 1e-12
    for k in range(6):
        col = lr[ok[:, k], k]
        assert abs(o.mu_y[k] - col.mean()) < 1e-9 and abs(o.sd_y[k] - col.std(ddof=1)) < 1e-9
        np.testing.assert_allclose(t[ok[:, k], k], (col - o.mu_y[k]) / o.sd_y[k], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(x, (np.log(EN) - o.mu_x) / o.sd_x, rtol=1e-6, atol=1e-6)
    assert np.all(ln[~ok] == -200.0)
    # standard errors of the ln values: relative batch-means errors (1 %)
    assert np.all(np.isnan(sig[~ok]))
    np.testing.assert_allclose(sig[ok], 0.01, rtol=1e-6)
