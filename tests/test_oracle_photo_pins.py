"""Pins of the photoionization oracle (arXiv:2110.14494 Sec. 2.4) against
what the mathematics fixes: the absorption distribution against numerical
quadrature of f(r) and its normalisation (Frullani's integral), the mean
absorption distance in closed form, isotropy of the directions, the photon
yield of the UV source term, the loss outside the box against the bounds the
distribution gives, and independence of the event order.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import photo as P

K1, K2 = 5.25e3, 3.0e5  # 1/m: absorption lengths 190 um and 3.3 um


def _box(n=64, dx=1e-5):
    return {"x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}, n


def _events(n, seed, w=1.0, half=3.2e-4):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 2 * half, size=(n, 3)).astype(np.float32)
    ww = np.full(n, w, np.float32) if np.isscalar(w) else np.asarray(w, np.float32)
    return pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), ww


@pytest.mark.parametrize("r", [3e-7, 3e-6, 3e-5, 3e-4, 3e-3])
def test_distribution_is_the_integral_of_the_absorption_function(r):
    q = quad(lambda s: float(P.absorption_pdf(s, K1, K2)), 0.0, r, limit=400, points=[r * 1e-4, r * 1e-2])[0]
    assert abs(float(P.absorption_cdf(r, K1, K2)) - q) < 1e-10


def test_absorption_function_is_normalised():
    # Frullani: int_0^inf (e^-as - e^-bs) / s ds = ln(b / a)
    f = lambda s: float(P.absorption_pdf(s, K1, K2))
    tot = (quad(f, 0.0, 1e-5, limit=400, points=[1e-8, 1e-6])[0] + quad(f, 1e-5, 1e-3, limit=400)[0]
           + quad(f, 1e-3, np.inf, limit=400)[0])
    assert abs(tot - 1.0) < 1e-8


def test_distance_inverts_the_distribution():
    U = np.array([1e-4, 0.01, 0.2, 0.5, 0.8, 0.99, 0.999999])
    r = P.absorption_distance(U, K1, K2)
    assert np.all(np.diff(r) > 0)
    assert np.max(np.abs(P.absorption_cdf(r, K1, K2) - U)) < 1e-13


def test_mean_distance_and_isotropy():
    # E[r] = int r f(r) dr = (1/k1 - 1/k2) / ln(k2/k1); E[r^2] = (1/k1^2 - 1/k2^2) / ln(k2/k1)
    # (distinct event positions: an event's photons are keyed by its position bits)
    # (events near the origin, the box centre, so that single precision
    # resolves the short distances too)
    n = 200_000
    grid, nc = _box(4096, 1e-5)
    half = nc * grid["dx"] / 2
    grid.update(x0=-half, y0=-half, z0=-half)
    x, y, z, w = _events(n, 1, w=1.0, half=1e-4)
    x, y, z = (a - np.float32(1e-4) for a in (x, y, z))  # distances beyond 10 mm: probability < 1e-20
    out = P.photoionize(x, y, z, w, grid, 1.0, K1, K2, 1.0, seed=11, step=0, nx=nc, ny=nc, nz=nc)
    assert out["photons"] == n and out["absorbed"] == n  # eta w / w_photon = 1 exactly, box much larger than 1/k1
    L = math.log(K2 / K1)
    m1 = (1 / K1 - 1 / K2) / L
    m2 = (1 / K1 ** 2 - 1 / K2 ** 2) / L
    d = out["dist"]
    sd = math.sqrt(m2 - m1 * m1)
    assert abs(d.mean() - m1) < 5 * sd / math.sqrt(n)
    e = out["event"]
    dv = np.stack([out["x"].astype(np.float64) - x[e], out["y"].astype(np.float64) - y[e],
                   out["z"].astype(np.float64) - z[e]], axis=1)
    far = out["dist"] > 1e-7  # resolved to 1e-4 and better
    dv = dv[far]
    u = dv / np.linalg.norm(dv, axis=1, keepdims=True)
    n = dv.shape[0]
    # isotropic: each component mean 0 (sd 1/sqrt(3)), second moment 1/3 (sd sqrt(4/45))
    assert np.all(np.abs(u.mean(axis=0)) < 5 / math.sqrt(3 * n))
    assert np.all(np.abs((u * u).mean(axis=0) - 1 / 3) < 5 * math.sqrt(4 / 45 / n))


def test_photon_yield_of_the_source_term():
    n = 100_000
    grid, nc = _box()
    x, y, z, _ = _events(n, 2)
    # integral lambda: the count is exact
    out = P.photoionize(x, y, z, np.full(n, 8.0, np.float32), grid, 0.25, K1, K2, 1.0, 5, 3, nc, nc, nc)
    assert out["photons"] == 2 * n
    # fractional lambda: floor plus a Bernoulli of the fraction (mean exact, variance f(1 - f) per event)
    w = np.random.default_rng(3).uniform(1.0, 50.0, n).astype(np.float32)
    eta = 0.0028846
    cnt, wph = P.photon_counts(w, eta, 1.0, 5, 3, x, y, z)
    lam = eta * w.astype(np.float64)
    assert np.all((cnt == np.floor(lam)) | (cnt == np.floor(lam) + 1))
    fr = lam - np.floor(lam)
    assert abs(cnt.sum() - lam.sum()) < 5 * math.sqrt(np.sum(fr * (1 - fr)))
    assert np.all(wph == 1.0)
    # photons of the event's weight: Bernoulli(eta) per event
    cnt2, wph2 = P.photon_counts(w, 0.3, 0.0, 5, 3, x, y, z)
    assert set(np.unique(cnt2)) <= {0, 1}
    assert abs(cnt2.mean() - 0.3) < 5 * math.sqrt(0.21 / n)
    assert np.array_equal(wph2, w.astype(np.float64))


def test_loss_outside_the_box_is_bounded_by_the_distribution():
    # events at the centre of a cube of half-width a: a photon absorbed within
    # a stays inside, one beyond a sqrt(3) leaves
    n = 100_000
    dx, nc = 2e-6, 20
    grid = {"x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}
    a = nc * dx / 2
    rng = np.random.default_rng(4)
    x, y, z = (np.float32(a) + rng.uniform(-1e-9, 1e-9, n).astype(np.float32) for _ in range(3))
    w = np.ones(n, np.float32)
    out = P.photoionize(x, y, z, w, grid, 1.0, K1, K2, 1.0, 9, 0, nc, nc, nc)
    frac = out["absorbed"] / out["photons"]
    lo, hi = float(P.absorption_cdf(a, K1, K2)), float(P.absorption_cdf(a * math.sqrt(3), K1, K2))
    s = 5 * math.sqrt(0.25 / n)
    assert lo - s < frac < hi + s
    assert 0.05 < lo < hi < 0.95  # the case discriminates
    for c in ("x", "y", "z"):
        assert np.all((out[c] >= 0.0) & (out[c].astype(np.float64) < nc * dx))


def test_photons_do_not_depend_on_event_order():
    n = 5000
    grid, nc = _box()
    x, y, z, _ = _events(n, 5)
    w = np.random.default_rng(6).uniform(1, 400, n).astype(np.float32)
    a = P.photoionize(x, y, z, w, grid, 0.01, K1, K2, 1.0, 21, 7, nc, nc, nc)
    perm = np.random.default_rng(7).permutation(n)
    b = P.photoionize(x[perm], y[perm], z[perm], w[perm], grid, 0.01, K1, K2, 1.0, 21, 7, nc, nc, nc)
    ia, ib = np.argsort(a["id"]), np.argsort(b["id"])
    assert a["absorbed"] > 1000
    for k in ("id", "x", "y", "z", "w"):
        assert np.array_equal(a[k][ia], b[k][ib])
    # another step draws other photons
    c = P.photoionize(x, y, z, w, grid, 0.01, K1, K2, 1.0, 21, 8, nc, nc, nc)
    assert len(np.intersect1d(a["id"], c["id"])) == 0
