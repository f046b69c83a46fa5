"""Seeded synthetic inputs for the PIC-MCC electron update and the swarms.

This module only builds input arrays (particles, fields, cross sections and
E/N lists) with NumPy's seeded generators.  It holds none of the method's
arithmetic and serves the HIP library and the CPU oracle alike.

The paper's own inputs are Phelps' N2/O2 cross sections and streamer fields
of 15-190 kV/cm in air at 1 bar (arXiv:2110.14494, Sec. 2.1.5, Sec. 2.3,
Sec. 3.1); neither the cross-section data nor the streamer fields are
available here, so air-like synthetic stand-ins of the same shape are used:
  * gas: 80/20 N2/O2 mean molecular mass 28.81 u, N = 2.45e25 m^-3;
  * cross sections on 1000 log-spaced energies over 0.01-1000 eV: elastic
    6e-20 m^2; excitation 3e-21 m^2 above 11 eV; ionization
    2e-20 (1-15.6/eps) ln(eps/15.6)/(eps/15.6) m^2 above 15.6 eV; attachment
    1e-22 m^2 below 1 eV;
  * fields: uniform, or a background plus a Gaussian tip enhancement.
"""
from __future__ import annotations

import numpy as np

ELEMENTARY_CHARGE = 1.602176634e-19  # C
ELECTRON_MASS = 9.1093837015e-31  # kg
ATOMIC_MASS = 1.66053906660e-27  # kg
AIR_MASS = 28.81 * ATOMIC_MASS  # 0.8 N2 + 0.2 O2
GAS_N = 2.45e25  # m^-3
PAPER_GAS_N = 2.414e25  # m^-3, 1 bar and 300 K

ELASTIC, EXCITATION, IONIZATION, ATTACHMENT = 0, 1, 2, 3


def electron_species(gas_N: float = GAS_N, target_mass: float = AIR_MASS) -> dict:
    return {"mass": ELECTRON_MASS, "charge": -ELEMENTARY_CHARGE, "gas_N": gas_N,
            "target_mass": target_mass}


def node_energies(n_e: int, eps_min: float, eps_max: float) -> np.ndarray:
    """Log-spaced table energies eps_i = eps_min (eps_max/eps_min)^(i/(n_e-1))."""
    return eps_min * (eps_max / eps_min) ** (np.arange(n_e) / (n_e - 1))


def air_like_tables(n_e: int = 1000, eps_min: float = 0.01, eps_max: float = 1000.0) -> dict:
    eps = node_energies(n_e, eps_min, eps_max)
    s_el = np.full(n_e, 6e-20)
    s_exc = np.where(eps >= 11.0, 3e-21, 0.0)
    r = eps / 15.6
    with np.errstate(divide="ignore", invalid="ignore"):
        s_ion = np.where(eps >= 15.6, 2e-20 * (1.0 - 1.0 / r) * np.log(r) / r, 0.0)
    s_att = np.where(eps < 1.0, 1e-22, 0.0)
    return {"eps_min": eps_min, "eps_max": eps_max,
            "kind": np.array([ELASTIC, EXCITATION, IONIZATION, ATTACHMENT], dtype=np.int32),
            "threshold": np.array([0.0, 11.0, 15.6, 0.0]),
            "sigma": np.stack([s_el, s_exc, s_ion, s_att]), "flags": 0}


def rate_tables(rates: dict, n_e: int = 64, eps_min: float = 1e-3, eps_max: float = 1e4) -> dict:
    """Energy-independent collision frequencies (1/s), e.g. {ELASTIC: 1e12}.

    Used with the RATES flag for closed-form checks."""
    kinds = sorted(rates)
    return {"eps_min": eps_min, "eps_max": eps_max, "kind": np.array(kinds, dtype=np.int32),
            "threshold": np.zeros(len(kinds)),
            "sigma": np.stack([np.full(n_e, float(rates[k])) for k in kinds]), "flags": 2}


def uniform_grid(n: int, dx: float, E=(0.0, 0.0, 0.0), x0: float = 0.0) -> dict:
    E4 = np.zeros((n, n, n, 4), dtype=np.float32)
    E4[..., 0], E4[..., 1], E4[..., 2] = E
    return {"E": E4, "x0": x0, "y0": x0, "z0": x0, "dx": dx}


def tip_grid(n: int, length: float, background: float, peak: float, sigma: float, tip) -> dict:
    """E_z = background + peak exp(-|r - tip|^2 / (2 sigma^2)) at cell centres."""
    dx = length / n
    c = (np.arange(n) + 0.5) * dx
    gx = np.exp(-((c - tip[0]) ** 2) / (2 * sigma ** 2))
    gy = np.exp(-((c - tip[1]) ** 2) / (2 * sigma ** 2))
    gz = np.exp(-((c - tip[2]) ** 2) / (2 * sigma ** 2))
    E4 = np.zeros((n, n, n, 4), dtype=np.float32)
    E4[..., 2] = (background + peak * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]).astype(np.float32)
    return {"E": E4, "x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}


def gaussian_particles(n: int, centre, sigma: float, seed: int, weight_seed: int | None = None,
                       log_weight_max: float = 0.0) -> dict:
    """Electrons at rest, positions ~ N(centre, sigma^2) per axis, ids 0..n-1.

    Weights are 1, or log-uniform in [1, e^log_weight_max) if log_weight_max > 0."""
    rng = np.random.default_rng(seed)
    pos = rng.standard_normal((3, n)) * sigma + np.asarray(centre, dtype=np.float64)[:, None]
    if log_weight_max > 0:
        wr = np.random.default_rng(weight_seed if weight_seed is not None else seed + 1)
        w = np.exp(wr.random(n) * log_weight_max)
    else:
        w = np.ones(n)
    z = np.zeros(n, dtype=np.float32)
    return {"x": pos[0].astype(np.float32), "y": pos[1].astype(np.float32),
            "z": pos[2].astype(np.float32), "vx": z.copy(), "vy": z.copy(), "vz": z.copy(),
            "w": w.astype(np.float32), "id": np.arange(n, dtype=np.uint64)}


def uniform_box_particles(n: int, lo: float, hi: float, speed: float, seed: int) -> dict:
    """Positions uniform in [lo, hi)^3, isotropic velocities of one speed."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(lo, hi, size=(3, n))
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0)
    v = (speed * d).astype(np.float32)
    return {"x": pos[0].astype(np.float32), "y": pos[1].astype(np.float32),
            "z": pos[2].astype(np.float32), "vx": v[0], "vy": v[1], "vz": v[2],
            "w": np.ones(n, dtype=np.float32), "id": np.arange(n, dtype=np.uint64)}


# --- the benchmark workloads -------------------------------------------------

def plain_swarm_config(n: int = 10_000, seed: int = 0) -> dict:
    """1e4 electrons at rest in a Gaussian blob (sigma 50 um) at the centre of a
    1.28 mm cube; uniform E = 2e6 V/m along z on 32^3 cells of 40 um; 1000
    steps of 1 ps."""
    L = 32 * 40e-6
    return {"name": "plain-swarm-1e4-32c", "species": electron_species(), "tables": air_like_tables(),
            "grid": uniform_grid(32, 40e-6, (0.0, 0.0, 2e6)),
            "parts": gaussian_particles(n, (L / 2,) * 3, 50e-6, seed=seed + 100),
            "dt": 1e-12, "n_steps": 1000, "seed": seed}


def streamer_config(n: int = 2 ** 24, grid_n: int = 256, length: float = 10e-3, background: float = 1.5e6,
                    peak: float = 1.5e7, dt: float = 2e-12, n_steps: int = 200, pos_seed: int = 2,
                    weight_seed: int = 3, seed: int = 0, tip_frac=(0.5, 0.5, 0.8)) -> dict:
    """Streamer-scale stage: 2^24 electrons ~ N(tip, 300 um), weights
    log-uniform in 1-64, 256^3 cells over a 10 mm cube, field 1.5e6 V/m plus a
    Gaussian tip of 1.5e7 V/m (sigma 200 um) at z = 8 mm; 200 steps of 2 ps."""
    tip = tuple(f * length for f in tip_frac)
    return {"name": f"streamer-2^{int(np.log2(n))}-{grid_n}c", "species": electron_species(),
            "tables": air_like_tables(),
            "grid": tip_grid(grid_n, length, background, peak, 200e-6, tip),
            "parts": gaussian_particles(n, tip, 300e-6, seed=pos_seed, weight_seed=weight_seed,
                                        log_weight_max=np.log(64.0)),
            "dt": dt, "n_steps": n_steps, "seed": seed}


def stress_config(background: float = 1.5e6, n: int = 2 ** 27, n_steps: int = 100) -> dict:
    """Large stress stage: 2^27 electrons on 512^3 cells of 20 um, tip field
    as the streamer stage at (0.5, 0.5, 0.8) of the cube, 100 steps of 1 ps."""
    cfg = streamer_config(n=n, grid_n=512, length=512 * 20e-6, background=background, dt=1e-12,
                          n_steps=n_steps, pos_seed=2, weight_seed=3, seed=0)
    cfg["name"] = f"stress-2^{int(np.log2(n))}-512c-bg{background / 1e6:g}MV/m"
    return cfg


def tip_block_config(m: int = 64, n: int = 4096) -> dict:
    """The streamer stage's tip field (256^3 cells over 10 mm) cut to the m^3
    block of its cells centred on the tip, with the stage's first n electrons
    (which start within a few sigma of the tip, inside the block)."""
    cfg = streamer_config(n=n)
    g = cfg["grid"]
    dx = g["dx"]
    ci = int(round(5e-3 / dx)) - m // 2
    ck = int(round(8e-3 / dx)) - m // 2
    E = np.ascontiguousarray(g["E"][ck:ck + m, ci:ci + m, ci:ci + m])
    cfg["grid"] = {"E": E, "x0": ci * dx, "y0": ci * dx, "z0": ck * dx, "dx": dx}
    cfg["name"] = f"tip-block-{m}c-n{n}"
    return cfg


def steep_field_grid(n: int = 48, dx: float = 4e-6) -> dict:
    """A field with steep gradients on cells of 4 um: E_z rises from 1e6 to
    6e7 V/m within a few cells around z = 0 (tanh profile of width 1.5 cells)
    and E_x varies as 2e7 sin(2 pi y / L) V/m; the cube is centred on 0."""
    zc = (np.arange(n) + 0.5) * dx - n * dx / 2
    E4 = np.zeros((n, n, n, 4), np.float32)
    E4[..., 2] = (1e6 + 5.9e7 * 0.5 * (1 + np.tanh(zc / (1.5 * dx))))[:, None, None]
    E4[..., 0] = (2e7 * np.sin(2 * np.pi * (np.arange(n) + 0.5) / n))[None, :, None]
    return {"E": E4, "x0": -n * dx / 2, "y0": -n * dx / 2, "z0": -n * dx / 2, "dx": dx}


def swarm_batch_config(n_swarms: int = 256, en_lo: float = 10.0, en_hi: float = 1000.0, seed: int = 1,
                       log2_lo: float = 12.0, log2_hi: float = 17.0, scale: float = 1.0) -> dict:
    """256 swarms at E/N log-spaced over 10-1000 Td, sizes log-uniform in
    2^12-2^17 (seed 1); 2000 steps of 1 ps, sampled every 10 steps."""
    EN = en_lo * (en_hi / en_lo) ** (np.arange(n_swarms) / max(n_swarms - 1, 1))
    rng = np.random.default_rng(seed)
    n0 = np.floor(2.0 ** (log2_lo + (log2_hi - log2_lo) * rng.random(n_swarms)) * scale)
    return {"EN_Td": EN, "n0": np.maximum(n0, 1).astype(np.int32), "dt": 1e-12, "n_steps": 2000,
            "sample_every": 10, "window_start": 500e-12, "seed": 0}


def log_uniform_EN(n: int, seed: int, lo: float = 10.0, hi: float = 1000.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (lo * (hi / lo) ** rng.random(n)).astype(np.float32)


def mlp_init(seed: int = 4) -> np.ndarray:
    """Initial surrogate parameters (Glorot-uniform weights, zero biases) in
    the packed order W1[64,1], b1[64], W2[64,64], b2[64], W3[6,64], b3[6],
    rounded to single precision; returned as float64."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((64, 1), (64,), (64, 64), (64,), (6, 64), (6,)):
        if len(shape) == 2:
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
