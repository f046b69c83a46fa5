"""Plain FP64 reference of the coefficient surrogate (test infrastructure).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The surrogate maps x = standardised ln(E/N) to six standardised log
coefficients (ln mobility N, ln D_L N, ln alpha/N, ln eta/N, ln mean energy,
ln W_bulk/W_flux) with a 1 -> 64 -> 64 -> 6 perceptron, tanh on the two
hidden layers and a linear output:
    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3.
Loss: mean squared error over the valid (unmasked) target entries,
    L = sum(mask * (y - t)^2) / sum(mask).
Parameters are packed in one vector in the order W1[64,1], b1[64],
W2[64,64], b2[64], W3[6,64], b3[6] (row-major), 4678 values.
Training: full-batch Adam (Kingma & Ba 2015) with a cosine learning-rate
schedule from lr0 to lr_min.
"""
from __future__ import annotations

import numpy as np

H = 64
NOUT = 6
SHAPES = (("W1", (H, 1)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (NOUT, H)), ("b3", (NOUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, x):
    """x [n] -> (y [n, 6], cache)."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 1)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, h1, h2)


def loss_and_grad(theta, x, t, mask):
    """Masked MSE and its gradient by explicit back-propagation."""
    p = unpack(theta)
    y, (xx, h1, h2) = forward(theta, x)
    m = np.asarray(mask, dtype=np.float64)
    cnt = m.sum()
    r = (y - t) * m
    L = np.sum(r * r) / cnt
    dy = 2.0 * r / cnt
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dz2 = (dy @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ xx
    g["b1"] = dz1.sum(0)
    return L, pack(g)


def loss_only(theta, x, t, mask):
    y, _ = forward(theta, x)
    m = np.asarray(mask, dtype=np.float64)
    r = (y - t) * m
    return np.sum(r * r) / m.sum()


def cosine_lr(epoch: int, epochs: int, lr0: float, lr_min: float) -> float:
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * epoch / epochs))


def train(theta0, x, t, mask, epochs: int, lr0: float, lr_min: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam; returns (theta, loss per epoch before the update)."""
    theta = np.array(theta0, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = np.empty(epochs)
    for e in range(epochs):
        L, g = loss_and_grad(theta, x, t, mask)
        losses[e] = L
        lr = cosine_lr(e, epochs, lr0, lr_min)
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** (e + 1))
        vh = v / (1 - beta2 ** (e + 1))
        theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, losses


def bf16_round(a):
    """Round to bfloat16 (nearest, ties to even) and back to float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, x):
    """The inference as the device computes it: weights rounded to bfloat16; a
    hidden activation tanh(z) carried as s = (1 + tanh z) / 2 (the logistic
    function of 2 z) and rounded to bfloat16 in that form, so the next layer
    sees 2 s - 1; products accumulated exactly (here in float64)."""
    p = unpack(theta)
    W1, b1, W2, b2, W3, b3 = (p[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    x = np.asarray(x, dtype=np.float64).reshape(-1, 1)
    h1 = 2.0 * bf16_round(0.5 * (1.0 + np.tanh(x @ W1.T + b1))) - 1.0
    h2 = 2.0 * bf16_round(0.5 * (1.0 + np.tanh(h1 @ bf16_round(W2).T + b2))) - 1.0
    return h2 @ bf16_round(W3).T + b3
