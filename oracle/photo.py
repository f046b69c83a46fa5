"""Discrete photoionization (arXiv:2110.14494 Sec. 2.4: Zheleznyak's model,
the UV source term eta = p_q / (p + p_q) xi photons per ionization,
isotropic photon directions, absorption function f(r), discrete photons).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product library.
Plain NumPy/SciPy in double precision, one definition at a time.

Readings where the paper is silent (the absorption constants are not given,
so they are inputs):
* f(r) = (exp(-k1 r) - exp(-k2 r)) / (r ln(k2 / k1)) with k1 = chi_min p_O2
  and k2 = chi_max p_O2 of Zheleznyak's model; its distribution function is
  F(r) = 1 - (E1(k1 r) - E1(k2 r)) / ln(k2 / k1) (E1 the exponential
  integral) and a distance solves F(r) = U, by 64 bisections on ln r over
  [ln(1e-6 / k2), ln(60 / k1)];
* an ionization event of weight w emits lambda = eta w / w_photon photons of
  weight w_photon (w_photon <= 0: photons of the event's weight, lambda =
  eta), floor(lambda) plus one more with probability lambda - floor(lambda);
* each photon flies in an isotropic direction (cos theta = 1 - 2 u, azimuth
  2 pi u') and leaves a photoelectron at rest plus a positive ion where it is
  absorbed; the point is rounded to single precision and the photon is lost
  if that point lies outside the grid box;
* random numbers: Philox4x32-10 with key (seed low ^ 0x50484F54, seed high ^
  step low) and counter (bit patterns of the event's x, y, z; c): c = 0 the
  count's uniform, c = 2j + 1 photon j's direction and distance, c = 2j + 2
  its id, so that an event's photons do not depend on its place in the list.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import exp1

from . import philox4x32_10

SALT = 0x50484F54


def absorption_pdf(r, k1: float, k2: float):
    """f(r), the probability density of the absorption distance."""
    r = np.asarray(r, dtype=np.float64)
    return (np.exp(-k1 * r) - np.exp(-k2 * r)) / (r * math.log(k2 / k1))


def absorption_cdf(r, k1: float, k2: float):
    """F(r) = 1 - (E1(k1 r) - E1(k2 r)) / ln(k2 / k1)."""
    r = np.asarray(r, dtype=np.float64)
    return 1.0 - (exp1(k1 * r) - exp1(k2 * r)) / math.log(k2 / k1)


def absorption_distance(U, k1: float, k2: float):
    """r with F(r) = U: 64 bisections on ln r."""
    U = np.asarray(U, dtype=np.float64)
    lo = np.full(U.shape, math.log(1e-6 / k2))
    hi = np.full(U.shape, math.log(60.0 / k1))
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = absorption_cdf(np.exp(mid), k1, k2) < U
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return np.exp(0.5 * (lo + hi))


def _key(seed: int, step: int) -> np.ndarray:
    return np.array([(seed & 0xFFFFFFFF) ^ SALT, ((seed >> 32) & 0xFFFFFFFF) ^ (step & 0xFFFFFFFF)], np.uint32)


def _draws(xb, yb, zb, c, key):
    ctr = np.stack([xb, yb, zb, np.asarray(c, np.uint32)], axis=1).astype(np.uint32)
    keys = np.broadcast_to(key, (ctr.shape[0], 2)).copy()
    return philox4x32_10(ctr, keys)


def _u32(r):
    return (r.astype(np.float64) + 0.5) * 2.0 ** -32


def photon_counts(ev_w, eta: float, w_photon: float, seed: int, step: int, ev_x, ev_y, ev_z):
    """(photons per event, photon weight per event)."""
    w = np.asarray(ev_w, np.float32).astype(np.float64)
    if w_photon > 0:
        lam = eta * w / w_photon
        wph = np.full(w.shape, float(w_photon))
    else:
        lam = np.full(w.shape, float(eta))
        wph = w
    xb, yb, zb = (np.asarray(a, np.float32).view(np.uint32) for a in (ev_x, ev_y, ev_z))
    n = np.zeros(w.shape, np.int64)
    if w.size == 0:
        return n, wph
    r = _draws(xb, yb, zb, np.zeros(w.size, np.uint32), _key(seed, step))
    fl = np.floor(lam)
    n = np.where(lam > 0, fl.astype(np.int64) + (_u32(r[:, 0]) < lam - fl), 0)
    return n, wph


def photoionize(ev_x, ev_y, ev_z, ev_w, grid: dict, eta: float, k1: float, k2: float, w_photon: float, seed: int,
                step: int, nx: int, ny: int, nz: int):
    """Photoelectrons of the events: dict with x, y, z (float32), w
    (float32), id (uint64) of those absorbed inside the box, and counts
    photons / absorbed."""
    ev_x, ev_y, ev_z = (np.asarray(a, np.float32) for a in (ev_x, ev_y, ev_z))
    cnt, wph = photon_counts(ev_w, eta, w_photon, seed, step, ev_x, ev_y, ev_z)
    e = np.repeat(np.arange(cnt.size), cnt)
    j = np.concatenate([np.arange(c) for c in cnt]) if cnt.size else np.zeros(0, np.int64)
    key = _key(seed, step)
    xb, yb, zb = (a.view(np.uint32)[e] for a in (ev_x, ev_y, ev_z))
    out = {"photons": int(cnt.sum())}
    if e.size == 0:
        out.update(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                   w=np.zeros(0, np.float32), id=np.zeros(0, np.uint64), absorbed=0)
        return out
    r = _draws(xb, yb, zb, (2 * j + 1).astype(np.uint32), key)
    q = _draws(xb, yb, zb, (2 * j + 2).astype(np.uint32), key)
    ct = 1.0 - 2.0 * _u32(r[:, 0])
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * _u32(r[:, 1])
    U = ((r[:, 2] >> 5).astype(np.float64) * 67108864.0 + (r[:, 3] >> 6).astype(np.float64) + 0.5) * 2.0 ** -53
    dist = absorption_distance(U, k1, k2)
    px = (ev_x[e].astype(np.float64) + dist * (st * np.cos(ph))).astype(np.float32)
    py = (ev_y[e].astype(np.float64) + dist * (st * np.sin(ph))).astype(np.float32)
    pz = (ev_z[e].astype(np.float64) + dist * ct).astype(np.float32)
    dx = float(grid["dx"])
    lo = (float(grid["x0"]), float(grid["y0"]), float(grid["z0"]))
    hi = (lo[0] + nx * dx, lo[1] + ny * dx, lo[2] + nz * dx)
    keep = np.ones(e.size, bool)
    for p, a, b in ((px, lo[0], hi[0]), (py, lo[1], hi[1]), (pz, lo[2], hi[2])):
        keep &= (p.astype(np.float64) >= a) & (p.astype(np.float64) < b)
    ids = q[:, 0].astype(np.uint64) | (q[:, 1].astype(np.uint64) << np.uint64(32))
    out.update(x=px[keep], y=py[keep], z=pz[keep], w=wph[e][keep].astype(np.float32), id=ids[keep],
               absorbed=int(keep.sum()), event=e[keep], dist=dist[keep])
    return out
