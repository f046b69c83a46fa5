"""Plain CPU oracle for the PIC-MCC electron update (arXiv:2110.14494, Sec. 2.1).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library: the particle update, the tables and the deposit are written in plain
double-precision C++ (``pcmcc_oracle.cpp``), the swarm estimators, the MLP,
the electrostatics and time step of the self-consistent step, the fluid step
and the discrete photoionization in NumPy/SciPy (``estimators.py``,
``mlp.py``, ``field.py``, ``fluid.py``, ``photo.py``).

This module only loads the compiled oracle (building it with g++ if needed)
and converts NumPy arrays to and from its C entry points.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcmcc_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

ELASTIC, EXCITATION, IONIZATION, ATTACHMENT = 0, 1, 2, 3
EFFECTIVE_TO_ELASTIC, RATES = 1, 2
STATS_FIELDS = ("n", "steps_done", "particle_steps", "trials", "null", "elastic",
                "excitation", "ionization", "attachment", "lost", "out_of_table", "errors",
                "majorant_violations", "bound_local", "bound_global")
N_MOMENTS = 14


def build(force: bool = False) -> str:
    """Compiles the oracle shared library (plain g++, OpenMP, no contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Problem(C.Structure):
    _fields_ = [("mass", C.c_double), ("charge", C.c_double), ("gas_N", C.c_double),
                ("target_mass", C.c_double), ("n_e", C.c_int), ("eps_min", C.c_double),
                ("eps_max", C.c_double), ("n_proc", C.c_int), ("kind", C.POINTER(C.c_int)),
                ("threshold", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
                ("flags", C.c_int)]


class Grid(C.Structure):
    _fields_ = [("E", C.POINTER(C.c_double)), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double), ("dx", C.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB_PATH)
            vp = C.c_void_p
            L.orc_philox4x32_10.argtypes = [vp, vp, vp, C.c_int64]
            L.orc_philox4x32_10.restype = None
            L.orc_set_constant_majorant.argtypes = [C.c_int]
            L.orc_set_constant_majorant.restype = None
            L.orc_set_majorant_fault.argtypes = [C.c_int]
            L.orc_set_majorant_fault.restype = None
            L.orc_build_tables.argtypes = [C.POINTER(Problem), vp, vp, vp, vp]
            L.orc_lookup.argtypes = [C.POINTER(Problem), C.c_int64, vp, vp, vp, vp]
            L.orc_pic_run.argtypes = [C.POINTER(Problem), C.POINTER(Grid)] + [vp] * 8 + [
                vp, C.c_int64, C.c_double, C.c_int, C.c_uint64, C.c_uint64, vp, C.c_int, C.c_double, C.c_double,
                vp, vp, vp, vp, C.c_int64, vp]
            L.orc_update_weights.argtypes = [vp] * 8 + [C.c_int64, C.c_int, C.c_int, C.c_int] + [C.c_double] * 5 + [
                C.c_uint64, C.c_uint64] + [vp] * 8 + [C.c_int64, vp, vp]
            L.orc_deposit.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int, C.c_int, C.c_int,
                                      C.c_double, C.c_double, C.c_double, C.c_double, vp]
            L.orc_swarm_run.argtypes = [C.POINTER(Problem), C.c_int, vp, vp, C.c_double, C.c_int,
                                        C.c_uint64, C.c_int, C.c_int64, C.c_int, vp, vp, vp, C.c_int]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the arrays a ctypes struct points to."""

    def __init__(self, *arrays):
        self.arrays = arrays


def make_problem(species: dict, tables: dict):
    """species: mass, charge, gas_N, target_mass; tables: eps_min, eps_max,
    kind[n_proc], threshold[n_proc], sigma[n_proc][n_e], flags."""
    kind = np.ascontiguousarray(tables["kind"], dtype=np.int32)
    thr = np.ascontiguousarray(tables["threshold"], dtype=np.float64)
    sig = np.ascontiguousarray(tables["sigma"], dtype=np.float64)
    pb = Problem(float(species["mass"]), float(species["charge"]), float(species["gas_N"]),
                 float(species["target_mass"]), int(sig.shape[1]), float(tables["eps_min"]),
                 float(tables["eps_max"]), int(sig.shape[0]),
                 kind.ctypes.data_as(C.POINTER(C.c_int)), thr.ctypes.data_as(C.POINTER(C.c_double)),
                 sig.ctypes.data_as(C.POINTER(C.c_double)), int(tables.get("flags", 0)))
    return pb, _Keep(kind, thr, sig)


def make_grid(grid: dict):
    """grid: E as float array [nz][ny][nx][3 or 4] (V/m), x0, y0, z0, dx."""
    E = np.ascontiguousarray(np.asarray(grid["E"])[..., :3], dtype=np.float64)
    nz, ny, nx = E.shape[:3]
    g = Grid(E.ctypes.data_as(C.POINTER(C.c_double)), nx, ny, nz, float(grid["x0"]),
             float(grid["y0"]), float(grid["z0"]), float(grid["dx"]))
    return g, _Keep(E)


def set_constant_majorant(on: bool) -> None:
    """Test knob: replace the majorant rule by the constant table maximum."""
    lib().orc_set_constant_majorant(1 if on else 0)


def set_majorant_fault(mode: int) -> None:
    """Test knob: plant a known mistake in the majorant rule (1: drop the
    field-range term of the speed bound, 2: nine tenths of every majorant;
    0: the rule as stated), to show that the violation counter catches it."""
    lib().orc_set_majorant_fault(int(mode))


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr [n,4] uint32, key [n,2] uint32 -> [n,4] uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(np.broadcast_to(np.asarray(key, dtype=np.uint32).reshape(-1, 2),
                                               (ctr.shape[0], 2)))
    out = np.empty_like(ctr)
    lib().orc_philox4x32_10(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0])
    return out


def build_tables(species: dict, tables: dict) -> dict:
    pb, keep = make_problem(species, tables)
    n, k = pb.n_e, pb.n_proc
    node = np.empty(n)
    nu = np.empty((k, n))
    Cc = np.empty((k, n))
    P = np.empty(n)
    rc = lib().orc_build_tables(C.byref(pb), _ptr(node), _ptr(nu), _ptr(Cc), _ptr(P))
    del keep
    if rc:
        raise ValueError(f"oracle build_tables failed ({rc})")
    return {"node": node, "nu": nu, "C": Cc, "P": P}


def lookup(species: dict, tables: dict, eps, s_ub=None):
    """Interpolated cumulative rates at eps [m] -> [m, n_proc]; with s_ub [m],
    also the collision-frequency majorant for those speed bounds."""
    pb, keep = make_problem(species, tables)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    m = eps.size
    cum = np.empty((m, pb.n_proc))
    maj = None
    if s_ub is not None:
        s_ub = np.ascontiguousarray(np.broadcast_to(s_ub, (m,)), dtype=np.float64)
        maj = np.empty(m)
        rc = lib().orc_lookup(C.byref(pb), m, _ptr(eps), _ptr(cum), _ptr(s_ub), _ptr(maj))
    else:
        rc = lib().orc_lookup(C.byref(pb), m, _ptr(eps), _ptr(cum), None, None)
    del keep
    if rc:
        raise ValueError(f"oracle lookup failed ({rc})")
    return cum, maj


def pic_run(species: dict, tables: dict, grid: dict, parts: dict, dt: float, n_steps: int,
            seed: int, step0: int = 0, capacity: int | None = None, n_threads: int = 0, n_ppc: float = 0.0,
            growth: float = 1.25, n_ref: int = 0, events: bool = False):
    """Runs the PIC-MCC update on a copy of `parts` (x, y, z, vx, vy, vz, w, id).

    With n_ppc > 0 the super-particle weights are updated whenever the count
    exceeds floor(growth * n_ref) after a step (n_ref = 0: the start count).
    Returns (rc, parts_out, stats) with parts_out in double precision; stats
    also holds weight_updates, merged_pairs, splits and n_ref, and with
    events=True the committed steps' ionization and attachment events as
    float32 arrays [k, 4] (x, y, z, w) under ion_events and att_events."""
    pb, k1 = make_problem(species, tables)
    g, k2 = make_grid(grid)
    n = int(np.asarray(parts["x"]).size)
    cap = int(capacity if capacity is not None else max(4 * n, 1024))
    arrs = {}
    for key in ("x", "y", "z", "vx", "vy", "vz", "w"):
        a = np.zeros(cap, dtype=np.float64)
        a[:n] = np.asarray(parts[key], dtype=np.float64)
        arrs[key] = a
    ids = np.zeros(cap, dtype=np.uint64)
    ids[:n] = np.asarray(parts["id"], dtype=np.uint64)
    n_io = C.c_int64(n)
    stats = np.zeros(len(STATS_FIELDS), dtype=np.int64)
    wstats = np.zeros(3, dtype=np.int64)
    nref = C.c_int64(int(n_ref))
    ev_cap = 2 * cap if events else 0
    ion = np.zeros((ev_cap, 4), dtype=np.float32)
    att = np.zeros((ev_cap, 4), dtype=np.float32)
    ev_n = np.zeros(2, dtype=np.int64)
    rc = lib().orc_pic_run(C.byref(pb), C.byref(g), *[_ptr(arrs[k]) for k in
                                                     ("x", "y", "z", "vx", "vy", "vz", "w")],
                           _ptr(ids), C.byref(n_io), cap, float(dt), int(n_steps), int(seed),
                           int(step0), _ptr(stats), int(n_threads), float(n_ppc), float(growth), C.byref(nref),
                           _ptr(wstats), _ptr(ion) if events else None, _ptr(att) if events else None, ev_cap,
                           _ptr(ev_n) if events else None)
    del k1, k2
    m = n_io.value
    out = {k: v[:m].copy() for k, v in arrs.items()}
    out["id"] = ids[:m].copy()
    st = dict(zip(STATS_FIELDS, (int(s) for s in stats)))
    st.update(weight_updates=int(wstats[0]), merged_pairs=int(wstats[1]), splits=int(wstats[2]), n_ref=nref.value)
    if events:
        st["ion_events"] = ion[:min(int(ev_n[0]), ev_cap)].copy()
        st["att_events"] = att[:min(int(ev_n[1]), ev_cap)].copy()
    return rc, out, st


def update_weights(parts: dict, grid: dict, n_ppc: float, seed: int, update_index: int,
                   capacity: int | None = None):
    """Super-particle weight update (Sec. 2.1.2) of single-precision particle
    arrays on the grid; returns (rc, parts_out, counts) with counts =
    {merged_pairs, splits}."""
    n = int(np.asarray(parts["x"]).size)
    cap = int(capacity if capacity is not None else 2 * n + 16)
    ins = [np.ascontiguousarray(parts[k], dtype=np.float32) for k in ("x", "y", "z", "vx", "vy", "vz", "w")]
    ids = np.ascontiguousarray(parts["id"], dtype=np.uint64)
    outs = [np.zeros(cap, dtype=np.float32) for _ in range(7)]
    oid = np.zeros(cap, dtype=np.uint64)
    E = np.asarray(grid["E"])
    nz, ny, nx = E.shape[:3]
    n_out = C.c_int64(0)
    counts = np.zeros(2, dtype=np.int64)
    rc = lib().orc_update_weights(*[_ptr(a) for a in ins], _ptr(ids), n, nx, ny, nz, float(grid["x0"]),
                                  float(grid["y0"]), float(grid["z0"]), float(grid["dx"]), float(n_ppc), int(seed),
                                  int(update_index), *[_ptr(a) for a in outs], _ptr(oid), cap, C.byref(n_out),
                                  _ptr(counts))
    m = min(n_out.value, cap)
    out = {k: a[:m].copy() for k, a in zip(("x", "y", "z", "vx", "vy", "vz", "w"), outs)}
    out["id"] = oid[:m].copy()
    return rc, out, {"merged_pairs": int(counts[0]), "splits": int(counts[1])}


def deposit_rc(x, y, z, w, grid: dict):
    """Fixed-point CIC deposit of single-precision particle arrays; returns
    (rc, rho).  rc = -8 (rho all zero) if a weight is outside [0, 2^31) or a
    cell's exact sum leaves the int64 range."""
    x, y, z, w = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z, w))
    E = np.asarray(grid["E"])
    nz, ny, nx = E.shape[:3]
    rho = np.zeros((nz, ny, nx), dtype=np.int64)
    inv_dx = 1.0 / float(grid["dx"])
    rc = lib().orc_deposit(_ptr(x), _ptr(y), _ptr(z), _ptr(w), x.size, nx, ny, nz, float(grid["x0"]),
                           float(grid["y0"]), float(grid["z0"]), inv_dx, _ptr(rho))
    return rc, rho


def deposit(x, y, z, w, grid: dict) -> np.ndarray:
    """Fixed-point CIC deposit of single-precision particle arrays."""
    rc, rho = deposit_rc(x, y, z, w, grid)
    if rc != 0:
        raise ValueError(f"deposit out of the fixed-point range (rc {rc})")
    return rho


def swarm_run(species: dict, tables: dict, EN_Td, n0, dt: float, n_steps: int, seed: int,
              sample_every: int, cap_factor: int = 8, n_threads: int = 0, population_control: bool = True):
    """Uniform-field swarms; returns (rc, moments[S,J,14], counters[S,J,4], stats)."""
    pb, keep = make_problem(species, tables)
    EN = np.ascontiguousarray(EN_Td, dtype=np.float64)
    n0 = np.ascontiguousarray(n0, dtype=np.int32)
    S = EN.size
    J = n_steps // sample_every
    mom = np.zeros((S, J, N_MOMENTS))
    cnt = np.zeros((S, J, 4), dtype=np.int64)
    stats = np.zeros(len(STATS_FIELDS), dtype=np.int64)
    rc = lib().orc_swarm_run(C.byref(pb), S, _ptr(EN), _ptr(n0), float(dt), int(n_steps), int(seed),
                             int(sample_every), int(cap_factor), 1 if population_control else 0, _ptr(mom),
                             _ptr(cnt), _ptr(stats), int(n_threads))
    del keep
    return rc, mom, cnt, dict(zip(STATS_FIELDS, (int(s) for s in stats)))
