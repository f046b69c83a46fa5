"""Pins of the FP64 surrogate reference (CPU): explicit back-propagation
against central finite differences and against torch's FP64 autograd; the
bfloat16 rounding against known values; Adam training on a smooth target."""
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


def test_bf16_emulation_without_rounding_is_the_network(monkeypatch):
    # The emulation carries each hidden activation as s = (1 + tanh z) / 2 and
    # feeds 2 s - 1 on; with the rounding switched off that is the network
    # itself (the same output to rounding).
    rng = np.random.default_rng(11)
    th = W.mlp_init(7) + rng.normal(0, 0.3, M.N_PARAMS)
    x = rng.uniform(-3, 3, 400)
    monkeypatch.setattr(M, "bf16_round", lambda a: np.asarray(a, dtype=np.float64))
    y_em = M.forward_bf16(th, x)
    y_ref, _ = M.forward(th, x)
    np.testing.assert_allclose(y_em, y_ref, rtol=0, atol=1e-12)


def test_bf16_emulation_within_its_rounding_bound():
    # Rounding to bfloat16 moves a value by at most 2^-8 of itself; the bound
    # follows that through the two hidden layers (tanh and the logistic
    # function change by no more than their argument) and the output layer.
    rng = np.random.default_rng(12)
    th = W.mlp_init(8) + rng.normal(0, 0.3, M.N_PARAMS)
    x = rng.uniform(-3, 3, 2000)
    y_em = M.forward_bf16(th, x)
    y_ref, _ = M.forward(th, x)
    p = M.unpack(th)
    u = 2.0 ** -8
    h1 = np.tanh(x.reshape(-1, 1) @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    d_h1 = 2 * u  # h = 2 s - 1 with s in (0, 1)
    aW2 = np.abs(p["W2"])
    d_z2 = (aW2.sum(axis=1) * (1 + u) * d_h1)[None, :] + u * (np.abs(h1) @ aW2.T)
    d_h2 = d_z2 + 2 * u
    aW3 = np.abs(p["W3"])
    bound = (1 + u) * (d_h2 @ aW3.T) + u * (np.abs(h2) @ aW3.T)
    err = np.abs(y_em - y_ref)
    assert np.all(err <= bound + 1e-12)
    # and the rounding does show (the emulation is not the exact network)
    assert err.max() > 1e-4
