"""Drift-diffusion-reaction fluid step with the local field approximation
(arXiv:2110.14494 Sec. 2.2: the electron density equation, Koren-limited
advective fluxes with central diffusive fluxes, Heun's method and the fluid
time-step limits; transport data versus E/N as in Sec. 2.2.2).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product library.
Plain NumPy in double precision, one step of the definitions at a time.

Readings where the paper is silent or garbled:
* electrons drift with v = -mu E; the electron flux is v n - D grad n and
  dn_e/dt = -div(flux) + (alpha - eta) mu |E| n_e; positive ions gain
  alpha mu |E| n_e and negative ions eta mu |E| n_e; ions do not move;
  photoionization is not part of this step;
* D is the longitudinal diffusion coefficient of the transport table;
* transport data are tables of mu N, D N, alpha / N, eta / N on log-spaced E/N
  nodes, interpolated linearly in ln(E/N) and held constant outside;
* face values: the field at a face is the mean of the two cells' field
  vectors; mu and D come from its magnitude; the normal velocity is -mu times
  its normal component;
* the advected face density is the upwind cell's value plus half the Koren
  limited slope, limiter psi(r) = max(0, min(2r, (1 + 2r) / 3, 2)) applied in
  slope form (no division); the diffusive flux is -D (n_R - n_L) / dx;
* homogeneous Neumann boundaries for the densities (Sec. 2.3) as mirror ghost
  cells (n_-1 = n_0, n_-2 = n_1); the field of a ghost cell is that of the
  boundary cell;
* the cell source uses the cell's field magnitude;
* Heun's method with the field recomputed (Poisson, Sec. 2.5) for the
  predicted densities; the time step is taken at the start of the step:
  dt = min(dt_max, 0.9 min(dt_cfl, dt_drt)) with
  dt_cfl = 0.5 / max over cells of (2 N_dim D / dx^2 + sum_i |v_i| / dx) (the
  printed limit drops D from the diffusion term) and
  dt_drt = eps0 / max over cells of (e n_e mu_e).
"""
from __future__ import annotations

import math

import numpy as np

from . import field as F

NDIM = 3


def table_eval(EN_Td, tab: dict, key: str) -> np.ndarray:
    """Linear interpolation in ln(E/N) on the table's log-spaced nodes, held
    constant outside; E/N = 0 takes the first node."""
    vals = np.asarray(tab[key], dtype=np.float64)
    n = vals.size
    lo, hi = math.log(tab["EN_lo"]), math.log(tab["EN_hi"])
    en = np.maximum(np.asarray(EN_Td, dtype=np.float64), 1e-300)
    u = (np.log(en) - lo) / (hi - lo) * (n - 1)
    u = np.clip(u, 0.0, n - 1.0)
    i = np.minimum(np.floor(u).astype(np.int64), n - 2)
    f = u - i
    return (1.0 - f) * vals[i] + f * vals[i + 1]


def koren(a, b):
    """Koren-limited slope from the upwind slope a and the downwind slope b:
    psi(b / a) a with psi(r) = max(0, min(2r, (1 + 2r) / 3, 2))."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    aa, ab = np.abs(a), np.abs(b)
    m = np.minimum(np.minimum(2.0 * ab, (aa + 2.0 * ab) / 3.0), 2.0 * aa)
    return np.where(a * b > 0, np.sign(a) * m, 0.0)


def _coefs(Emag, tab, gas_N):
    EN = Emag / gas_N * 1e21
    mu = table_eval(EN, tab, "muN") / gas_N
    D = table_eval(EN, tab, "DN") / gas_N
    alpha = table_eval(EN, tab, "alphaN") * gas_N
    eta = table_eval(EN, tab, "etaN") * gas_N
    return mu, D, alpha, eta


def derivatives(n_e, E, dx, tab, gas_N):
    """(dn_e/dt, dn_+/dt, dn_-/dt) on the cell centres for electron density
    n_e [nz][ny][nx] and cell field E [nz][ny][nx][3] (V/m)."""
    n = np.asarray(n_e, dtype=np.float64)
    Ec = np.asarray(E, dtype=np.float64)[..., :3]
    div = np.zeros_like(n)
    for ax in range(3):  # array axis: x -> 2, y -> 1, z -> 0
        arr_ax = 2 - ax
        m = n.shape[arr_ax]
        # mirror ghosts: two on each side
        idx = np.concatenate([[1, 0], np.arange(m), [m - 1, m - 2]])
        idx = np.clip(idx, 0, m - 1)
        p = np.take(n, idx, axis=arr_ax)  # p[j] = n at cell j - 2
        eidx = np.concatenate([[0], np.arange(m), [m - 1]])
        pe = np.take(Ec, eidx, axis=arr_ax)  # pe[j] = E at cell j - 1 (ghost = boundary cell)
        # faces f = 0..m: between cells f-1 and f
        nLL = np.take(p, np.arange(0, m + 1), axis=arr_ax)      # cell f-2
        nL = np.take(p, np.arange(1, m + 2), axis=arr_ax)       # cell f-1
        nR = np.take(p, np.arange(2, m + 3), axis=arr_ax)       # cell f
        nRR = np.take(p, np.arange(3, m + 4), axis=arr_ax)      # cell f+1
        EL = np.take(pe, np.arange(0, m + 1), axis=arr_ax)
        ER = np.take(pe, np.arange(1, m + 2), axis=arr_ax)
        Ef = 0.5 * (EL + ER)
        Efm = np.sqrt(np.sum(Ef * Ef, axis=-1))
        mu_f, D_f, _, _ = _coefs(Efm, tab, gas_N)
        v = -mu_f * Ef[..., ax]
        up = np.where(v >= 0, nL + 0.5 * koren(nL - nLL, nR - nL), nR + 0.5 * koren(nR - nRR, nL - nR))
        flux = v * up - D_f * (nR - nL) / dx
        div += (np.take(flux, np.arange(1, m + 1), axis=arr_ax) - np.take(flux, np.arange(0, m), axis=arr_ax)) / dx
    Em = np.sqrt(np.sum(Ec * Ec, axis=-1))
    mu_c, _, alpha, eta = _coefs(Em, tab, gas_N)
    rate = mu_c * Em * n
    return -div + (alpha - eta) * rate, alpha * rate, eta * rate


def time_step(n_e, E, dx, tab, gas_N, dt_max):
    """dt = min(dt_max, 0.9 min(dt_cfl, dt_drt)) at the state (n_e, E)."""
    Ec = np.asarray(E, dtype=np.float64)[..., :3]
    Em = np.sqrt(np.sum(Ec * Ec, axis=-1))
    mu, D, _, _ = _coefs(Em, tab, gas_N)
    cfl = 2 * NDIM * D / (dx * dx) + (mu * (np.abs(Ec[..., 0]) + np.abs(Ec[..., 1]) + np.abs(Ec[..., 2]))) / dx
    drt = F.QE * np.asarray(n_e, dtype=np.float64) * mu / F.EPS0
    c, d = float(cfl.max()), float(drt.max())
    dt_cfl = 0.5 / c if c > 0 else math.inf
    dt_drt = 1.0 / d if d > 0 else math.inf
    return min(dt_max, 0.9 * min(dt_cfl, dt_drt))


def charge(n_pos, n_e, n_neg):
    return ((np.asarray(n_pos, np.float64) - np.asarray(n_e, np.float64)) - np.asarray(n_neg, np.float64)) * F.QE


def fluid_run(grid: dict, n_e, n_pos, n_neg, tab: dict, gas_N: float, n_steps: int, dt_max: float):
    """n_steps Heun steps of the fluid model in the applied field of `grid`
    plus the space-charge field (Poisson with the boundary conditions of
    oracle.field).  Returns (n_e, n_pos, n_neg, info) with info: dt per step,
    the final field E and potential phi."""
    dx = float(grid["dx"])
    Ea = np.asarray(grid["E"], dtype=np.float32)[..., :3]
    ne, npo, nne = (np.asarray(a, dtype=np.float64).copy() for a in (n_e, n_pos, n_neg))

    def fld(a, b, c):
        phi = F.poisson(charge(b, a, c), dx)
        return phi, F.field(phi, Ea, dx)

    dts = []
    phi, E = fld(ne, npo, nne)
    for _ in range(n_steps):
        dt = time_step(ne, E, dx, tab, gas_N, dt_max)
        k1 = derivatives(ne, E, dx, tab, gas_N)
        s = (ne + dt * k1[0], npo + dt * k1[1], nne + dt * k1[2])
        _, Es = fld(*s)
        k2 = derivatives(s[0], Es, dx, tab, gas_N)
        ne = ne + 0.5 * dt * (k1[0] + k2[0])
        npo = npo + 0.5 * dt * (k1[1] + k2[1])
        nne = nne + 0.5 * dt * (k1[2] + k2[2])
        dts.append(dt)
        phi, E = fld(ne, npo, nne)
    return ne, npo, nne, {"dt": dts, "E": E, "phi": phi}
