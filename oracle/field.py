"""Electrostatics and time step of the self-consistent particle step
(arXiv:2110.14494: Sec. 2.5 Poisson's equation and E = -grad phi, Sec. 2.3
boundary conditions and ion seed, Sec. 2.1.4 time step).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product library.
Plain NumPy/SciPy in double precision, written from the definitions:

* The caller's field is the applied field (it stands in for the electrode and
  the applied voltage).  The space charge adds the potential phi of the
  discrete Poisson problem with phi = 0 on the two z faces (Dirichlet) and
  zero normal derivative on the x and y faces (homogeneous Neumann), Sec. 2.3;
  the electron update then sees E = E_applied - grad phi.
* Poisson's equation is read as lap phi = -rho / eps0 (the printed form drops
  the minus sign).
* Discretisation: the 7-point Laplacian on cell centres, the boundary
  conditions through ghost cells (Dirichlet at the face: ghost = -phi of the
  boundary cell; Neumann: ghost = phi); grad phi at a centre by central
  differences with the same ghosts.  The solve here is exact for that linear
  system: it is diagonal in the cosine basis (DCT-II) along x and y and the
  sine basis (DST-II) along z, with the eigenvalues of the 3-point operator.
* rho = e (n_+ - n_e - n_-) with each density the fixed-point CIC cell sum
  (2^-32 electrons) divided by the cell volume; ions do not move; an
  ionization adds a positive ion at the newborn's position, an attachment a
  negative ion where the electron was attached.
* Time step (Sec. 2.1.4): dt = min(dt_max, dt_cfl, dt_drt, dt_growth) with
  dt_cfl = 0.5 dx / v90, v90 the speed of rank ceil(9N/10) among the N
  particles (speeds ordered by |v|^2 rounded to single precision); dt_drt =
  eps0 / (e n_e,max mu_e), n_e,max the largest cell density (first cell in
  x-fastest order on ties) and mu_e the mobility at that cell's reduced field
  from a table of mu N over log-spaced E/N (linear in ln E/N, clamped);
  dt_growth = dt ln(1.2) / ln(N_new / N_old) when the physical electron number
  (sum of weights) grew over the last step.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft

EPS0 = 8.8541878128e-12
QE = 1.602176634e-19


def charge_density(n_pos, n_e, n_neg, dx: float) -> np.ndarray:
    """Space charge (C/m^3) from the three int64 fixed-point grids [nz][ny][nx]."""
    diff = (np.asarray(n_pos).astype(np.float64) - np.asarray(n_e).astype(np.float64)) - \
        np.asarray(n_neg).astype(np.float64)
    return diff * (QE * 2.0 ** -32 / (dx * dx * dx))


def _eig(n: int, dx: float, dirichlet: bool) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    if dirichlet:
        k = k + 1.0
    return -4.0 / (dx * dx) * np.sin(np.pi * k / (2.0 * n)) ** 2


def poisson(q: np.ndarray, dx: float) -> np.ndarray:
    """phi [nz][ny][nx] with lap phi = -q / eps0 under the boundary conditions
    above (exact solution of the discrete system)."""
    f = -np.asarray(q, dtype=np.float64) / EPS0
    nz, ny, nx = f.shape
    F = sfft.dct(f, type=2, axis=2, norm="ortho")
    F = sfft.dct(F, type=2, axis=1, norm="ortho")
    F = sfft.dst(F, type=2, axis=0, norm="ortho")
    lam = (_eig(nz, dx, True)[:, None, None] + _eig(ny, dx, False)[None, :, None] +
           _eig(nx, dx, False)[None, None, :])
    P = F / lam
    P = sfft.idst(P, type=2, axis=0, norm="ortho")
    P = sfft.idct(P, type=2, axis=1, norm="ortho")
    return sfft.idct(P, type=2, axis=2, norm="ortho")


def _ghosts(phi: np.ndarray):
    """phi padded by one ghost layer on every face (Neumann in x, y; Dirichlet in z)."""
    p = np.pad(phi, ((0, 0), (1, 1), (1, 1)), mode="edge")
    return np.concatenate([-p[:1], p, -p[-1:]], axis=0)


def laplacian(phi: np.ndarray, dx: float) -> np.ndarray:
    """The 7-point operator with the ghost cells (for checks)."""
    g = _ghosts(phi)
    c = g[1:-1, 1:-1, 1:-1]
    return ((g[1:-1, 1:-1, 2:] - 2 * c + g[1:-1, 1:-1, :-2]) + (g[1:-1, 2:, 1:-1] - 2 * c + g[1:-1, :-2, 1:-1]) +
            (g[2:, 1:-1, 1:-1] - 2 * c + g[:-2, 1:-1, 1:-1])) / (dx * dx)


def field(phi: np.ndarray, E_applied: np.ndarray, dx: float) -> np.ndarray:
    """E = E_applied - grad phi at the centres, single precision [nz][ny][nx][3]."""
    g = _ghosts(phi)
    gx = (g[1:-1, 1:-1, 2:] - g[1:-1, 1:-1, :-2]) / (2 * dx)
    gy = (g[1:-1, 2:, 1:-1] - g[1:-1, :-2, 1:-1]) / (2 * dx)
    gz = (g[2:, 1:-1, 1:-1] - g[:-2, 1:-1, 1:-1]) / (2 * dx)
    Ea = np.asarray(E_applied, dtype=np.float64)[..., :3]
    return (Ea - np.stack([gx, gy, gz], axis=-1)).astype(np.float32)


def speed_key(vx, vy, vz) -> np.ndarray:
    """|v|^2 from single-precision components, summed (vx^2 + vy^2) + vz^2 in
    double and rounded to single precision."""
    a, b, c = (np.asarray(v, dtype=np.float32).astype(np.float64) for v in (vx, vy, vz))
    return ((a * a + b * b) + c * c).astype(np.float32)


def quantile_rank(n: int) -> int:
    """1-based rank of the 90 % quantile: ceil(9 n / 10)."""
    return (9 * n + 9) // 10


def v90(vx, vy, vz) -> float:
    """Speed at the 90 % quantile (0 for no particles)."""
    key = speed_key(vx, vy, vz)
    if key.size == 0:
        return 0.0
    return math.sqrt(float(np.sort(key)[quantile_rank(key.size) - 1]))


def mobility(EN_Td: float, mu: dict, gas_N: float) -> float:
    """mu_e (m^2/(V s)) at E/N from a table of mu N over log-spaced E/N nodes
    {"EN_lo", "EN_hi", "muN"} (linear in ln E/N, clamped)."""
    muN = np.asarray(mu["muN"], dtype=np.float64)
    if muN.size == 1:
        return float(muN[0]) / gas_N
    lo, hi = math.log(mu["EN_lo"]), math.log(mu["EN_hi"])
    u = (math.log(max(EN_Td, 1e-300)) - lo) / (hi - lo) * (muN.size - 1)
    u = min(max(u, 0.0), muN.size - 1.0)
    i = min(int(math.floor(u)), muN.size - 2)
    f = u - i
    return float((1.0 - f) * muN[i] + f * muN[i + 1]) / gas_N


def drt_inputs(n_e: np.ndarray, E: np.ndarray, dx: float):
    """(n_e,max in m^-3, |E| at that cell) from the fixed-point electron grid."""
    flat = np.asarray(n_e).reshape(-1)
    if flat.size == 0 or flat.max() <= 0:
        return 0.0, 0.0
    c = int(np.argmax(flat))  # first maximum in x-fastest order
    e = np.asarray(E, dtype=np.float32).reshape(-1, 3)[c].astype(np.float64)
    return float(flat[c]) * 2.0 ** -32 / (dx * dx * dx), math.sqrt(float(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]))


def next_dt(dt_prev: float, dx: float, v90_: float, ne_max: float, mu_e: float, n_old: float, n_new: float,
            dt_max: float, cfl: float = 0.5, growth_max: float = 1.2) -> float:
    """Sec. 2.1.4: the smallest of the limits (dt_max when none applies)."""
    dt = dt_max
    if v90_ > 0:
        dt = min(dt, cfl * dx / v90_)
    if ne_max > 0 and mu_e > 0:
        dt = min(dt, EPS0 / (QE * ne_max * mu_e))
    if n_old > 0 and n_new > n_old:
        dt = min(dt, dt_prev * math.log(growth_max) / math.log(n_new / n_old))
    return dt


def streamer_run(species: dict, tables: dict, grid: dict, parts: dict, n_pos, n_neg, dt0: float, n_steps: int,
                 seed: int, step0: int = 0, capacity: int | None = None, adaptive: bool = True,
                 dt_max: float | None = None, mu: dict | None = None, cfl: float = 0.5, growth_max: float = 1.2):
    """Self-consistent steps: field from the densities at the start of each
    step, one electron step (Sec. 2.1.1) with that field, ion densities updated
    from the step's events, then the next time step.  n_pos and n_neg are
    int64 grids [nz][ny][nx], updated in place.  Returns (rc, parts_out
    (single precision), info) with info: dt (per step), t, E (the last field),
    phi, n_e, per-step v90, ne_max, electrons."""
    import oracle
    dx = float(grid["dx"])
    E_app = np.asarray(grid["E"])[..., :3]
    cur = {k: np.asarray(v, dtype=np.float32).copy() for k, v in parts.items() if k != "id"}
    cur["id"] = np.asarray(parts["id"], dtype=np.uint64).copy()
    mu = mu or {"muN": np.array([0.0])}
    dt_max = dt_max if dt_max is not None else dt0

    def densities():
        n_e = oracle.deposit(cur["x"], cur["y"], cur["z"], cur["w"], grid)
        phi = poisson(charge_density(n_pos, n_e, n_neg, dx), dx)
        return n_e, phi, field(phi, E_app, dx)

    n_e, phi, E = densities()
    n_tot = float(np.sum(cur["w"], dtype=np.float64))
    dt = float(dt0)
    info = {"dt": [], "v90": [], "ne_max": [], "electrons": [n_tot]}
    rc = 0
    t = 0.0
    for s in range(n_steps):
        g = dict(grid, E=E)
        rc, out, st = oracle.pic_run(species, tables, g, cur, dt, 1, seed, step0=step0 + s, capacity=capacity,
                                     events=True)
        if rc:
            break
        cur = {k: out[k].astype(np.float32) for k in ("x", "y", "z", "vx", "vy", "vz", "w")}
        cur["id"] = out["id"]
        for ev, grid_ in ((st["ion_events"], n_pos), (st["att_events"], n_neg)):
            if ev.shape[0]:
                grid_ += oracle.deposit(ev[:, 0], ev[:, 1], ev[:, 2], ev[:, 3], grid)
        n_e, phi, E = densities()
        info["dt"].append(dt)
        t += dt
        n_new = float(np.sum(cur["w"], dtype=np.float64))
        vq = v90(cur["vx"], cur["vy"], cur["vz"])
        ne_max, e_at = drt_inputs(n_e, E, dx)
        mu_e = mobility(e_at / species["gas_N"] * 1e21, mu, species["gas_N"]) if ne_max > 0 else 0.0
        info["v90"].append(vq)
        info["ne_max"].append(ne_max)
        info["electrons"].append(n_new)
        if adaptive:
            dt = next_dt(dt, dx, vq, ne_max, mu_e, n_tot, n_new, dt_max, cfl, growth_max)
        n_tot = n_new
    info.update(t=t, E=E, phi=phi, n_e=n_e, next_dt=dt)
    return rc, cur, info
