"""Python-side handles for the C ABI: a context, device particle arrays and a
device field grid, all backed by PyTorch tensors (memory and streams only).

Every function forwards to libpcmcc.so; nothing here computes.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _binding as B

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "w")


def _dev(device) -> torch.device:
    d = torch.device(device) if not isinstance(device, torch.device) else device
    if d.type != "cuda":
        raise ValueError("pcmcc runs on a HIP device only")
    return d


class Particles:
    """Structure-of-arrays electrons on the device with room for `capacity`."""

    def __init__(self, capacity: int, device="cuda:0"):
        dev = _dev(device)
        self.capacity = int(capacity)
        self.t = {k: torch.zeros(self.capacity, dtype=torch.float32, device=dev) for k in FIELDS}
        self.t["id"] = torch.zeros(self.capacity, dtype=torch.int64, device=dev)
        self.n_dev = torch.zeros(1, dtype=torch.int64, device=dev)

    @classmethod
    def from_numpy(cls, parts: dict, capacity: int | None = None, device="cuda:0") -> "Particles":
        n = int(np.asarray(parts["x"]).size)
        p = cls(capacity if capacity is not None else max(n, 1), device)
        if n > p.capacity:
            raise ValueError("more particles than capacity")
        for k in FIELDS:
            p.t[k][:n] = torch.from_numpy(np.ascontiguousarray(parts[k], dtype=np.float32))
        p.t["id"][:n] = torch.from_numpy(np.ascontiguousarray(parts["id"], dtype=np.uint64).view(np.int64))
        p.n_dev.fill_(n)
        return p

    @property
    def n(self) -> int:
        return int(self.n_dev.item())

    def to_numpy(self) -> dict:
        n = self.n
        out = {k: self.t[k][:n].cpu().numpy() for k in FIELDS}
        out["id"] = self.t["id"][:n].cpu().numpy().view(np.uint64)
        return out

    def struct(self) -> B.pcmcc_particles:
        t = self.t
        return B.pcmcc_particles(*(t[k].data_ptr() for k in FIELDS), t["id"].data_ptr(), self.n_dev.data_ptr(),
                                 self.capacity)


class DeviceGrid:
    """Cell-centred field grid on the device (float4 per cell, x fastest)."""

    def __init__(self, grid: dict, device="cuda:0"):
        E = np.asarray(grid["E"], dtype=np.float32)
        if E.ndim != 4 or E.shape[3] not in (3, 4):
            raise ValueError("E must be [nz][ny][nx][3|4]")
        if E.shape[3] == 3:
            E = np.concatenate([E, np.zeros(E.shape[:3] + (1,), np.float32)], axis=3)
        self.E = torch.from_numpy(np.ascontiguousarray(E)).to(_dev(device))
        self.nz, self.ny, self.nx = E.shape[:3]
        self.x0, self.y0, self.z0, self.dx = (float(grid[k]) for k in ("x0", "y0", "z0", "dx"))

    def struct(self) -> B.pcmcc_grid:
        return B.pcmcc_grid(self.E.data_ptr(), self.nx, self.ny, self.nz, self.x0, self.y0, self.z0, self.dx)

    def zeros_rho(self) -> torch.Tensor:
        return torch.zeros((self.nz, self.ny, self.nx), dtype=torch.int64, device=self.E.device)


def _photo_opts(photo: dict):
    return B.pcmcc_photo_opts(float(photo["eta"]), float(photo["k1"]), float(photo["k2"]),
                              float(photo.get("w_photon", 0.0)))


class Context:
    """One library context on a device, issuing work on a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        torch.cuda.set_device(device)
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        B.check(B.lib().pcmcc_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if self.h:
            B.lib().pcmcc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def last_error(self) -> str:
        return B.lib().pcmcc_last_error(self.h).decode()

    def init_species(self, species: dict):
        B.check(B.lib().pcmcc_init_species(self.h, float(species["mass"]), float(species["charge"]),
                                           float(species["gas_N"]), float(species["target_mass"])), self.h)

    def init_tables(self, tables: dict) -> int:
        kind = np.ascontiguousarray(tables["kind"], dtype=np.int32)
        thr = np.ascontiguousarray(tables["threshold"], dtype=np.float64)
        sig = np.ascontiguousarray(tables["sigma"], dtype=np.float64)
        return B.lib().pcmcc_init_tables(self.h, int(sig.shape[1]), float(tables["eps_min"]),
                                         float(tables["eps_max"]), int(sig.shape[0]),
                                         kind.ctypes.data_as(C.c_void_p), thr.ctypes.data_as(C.c_void_p),
                                         sig.ctypes.data_as(C.c_void_p), int(tables.get("flags", 0)))

    def setup(self, species: dict, tables: dict):
        self.init_species(species)
        B.check(self.init_tables(tables), self.h)

    def push_collide_deposit(self, parts: Particles, grid: DeviceGrid, dt: float, n_steps: int, seed: int,
                             step0: int = 0, rho: torch.Tensor | None = None, check: bool = True):
        st = B.pcmcc_stats()
        ps, gs = parts.struct(), grid.struct()
        rc = B.lib().pcmcc_push_collide_deposit(self.h, C.byref(ps), C.byref(gs), float(dt), int(n_steps),
                                                int(seed), int(step0),
                                                C.c_void_p(rho.data_ptr() if rho is not None else 0),
                                                C.byref(st))
        if check:
            B.check(rc, self.h)
        return rc, st.as_dict()

    def set_schedule(self, block: int = 0, blocks_per_cu: int = 0, refill_min: int = 0, chunk: int = 0):
        """Schedule of later step calls (pcmcc_set_schedule); zeros take the defaults."""
        s = B.pcmcc_schedule(int(block), int(blocks_per_cu), int(refill_min), int(chunk))
        B.check(B.lib().pcmcc_set_schedule(self.h, C.byref(s)), self.h)

    def get_schedule(self) -> dict:
        """The resolved schedule of the next step call (pcmcc_get_schedule)."""
        s = B.pcmcc_schedule()
        B.check(B.lib().pcmcc_get_schedule(self.h, C.byref(s)), self.h)
        return s.as_dict()

    def autotune_steps(self, parts: Particles, grid: DeviceGrid, dt: float, n_steps: int, seed: int, step0: int = 0,
                       tune_cache: str | None = None, check: bool = True):
        """Launch-shape tuner of the step kernel (pcmcc_autotune_steps): returns
        (rc, chosen schedule, tuned ms, default ms); parts is left unchanged."""
        ps, gs = parts.struct(), grid.struct()
        s = B.pcmcc_schedule()
        t_ms, d_ms = C.c_float(0), C.c_float(0)
        rc = B.lib().pcmcc_autotune_steps(self.h, C.byref(ps), C.byref(gs), float(dt), int(n_steps), int(seed),
                                          int(step0), tune_cache.encode() if tune_cache else None, C.byref(s),
                                          C.byref(t_ms), C.byref(d_ms))
        if check:
            B.check(rc, self.h)
        return rc, s.as_dict(), t_ms.value, d_ms.value

    def set_weight_control(self, n_ppc: float, growth: float = 1.25):
        B.check(B.lib().pcmcc_set_weight_control(self.h, float(n_ppc), float(growth)), self.h)

    def update_weights(self, parts: Particles, grid: DeviceGrid, n_ppc: float, seed: int, update_index: int,
                       check: bool = True):
        ps, gs = parts.struct(), grid.struct()
        mp, sp = C.c_int64(0), C.c_int64(0)
        rc = B.lib().pcmcc_update_weights(self.h, C.byref(ps), C.byref(gs), float(n_ppc), int(seed),
                                          int(update_index), C.byref(mp), C.byref(sp))
        if check:
            B.check(rc, self.h)
        return rc, {"merged_pairs": mp.value, "splits": sp.value}

    def deposit(self, parts: Particles, grid: DeviceGrid, rho: torch.Tensor, check: bool = True,
                no_alloc: bool = False) -> int:
        """Adds the particles' charge to rho (pcmcc_deposit, or with no_alloc
        pcmcc_deposit_noalloc, which allocates nothing and takes at most 2^21
        particles)."""
        t = parts.t
        gs = grid.struct()
        fn = B.lib().pcmcc_deposit_noalloc if no_alloc else B.lib().pcmcc_deposit
        rc = fn(self.h, t["x"].data_ptr(), t["y"].data_ptr(), t["z"].data_ptr(), t["w"].data_ptr(),
                parts.n_dev.data_ptr(), C.byref(gs), rho.data_ptr())
        if check:
            B.check(rc, self.h)
        return rc

    # --- self-consistent step -------------------------------------------------

    def solve_potential(self, grid: DeviceGrid, n_pos: torch.Tensor, n_e: torch.Tensor, n_neg: torch.Tensor,
                        phi: torch.Tensor, tol: float = 1e-10, max_cycles: int = 50):
        """Multigrid solve into phi (float64 [nz][ny][nx], also the start value);
        returns (cycles, relative residual)."""
        for t in (n_pos, n_e, n_neg):
            assert t.dtype == torch.int64 and t.is_contiguous() and t.numel() == grid.nx * grid.ny * grid.nz
        assert phi.dtype == torch.float64 and phi.is_contiguous() and phi.numel() == grid.nx * grid.ny * grid.nz
        cyc, rel = C.c_int(0), C.c_double(0)
        gs = grid.struct()
        B.check(B.lib().pcmcc_solve_potential(self.h, C.byref(gs), n_pos.data_ptr(), n_e.data_ptr(), n_neg.data_ptr(),
                                              phi.data_ptr(), float(tol), int(max_cycles), C.byref(cyc),
                                              C.byref(rel)), self.h)
        return cyc.value, rel.value

    def field_from_potential(self, grid: DeviceGrid, phi: torch.Tensor) -> torch.Tensor:
        """E_applied - grad phi as float32 [nz][ny][nx][4]."""
        assert phi.dtype == torch.float64 and phi.is_contiguous() and phi.numel() == grid.nx * grid.ny * grid.nz
        out = torch.empty((grid.nz, grid.ny, grid.nx, 4), dtype=torch.float32, device=grid.E.device)
        gs = grid.struct()
        B.check(B.lib().pcmcc_field_from_potential(self.h, C.byref(gs), phi.data_ptr(), out.data_ptr()), self.h)
        return out

    def speed_quantile(self, parts: Particles) -> float:
        v = C.c_double(0)
        t = parts.t
        B.check(B.lib().pcmcc_speed_quantile(self.h, t["vx"].data_ptr(), t["vy"].data_ptr(), t["vz"].data_ptr(),
                                             parts.n_dev.data_ptr(), C.byref(v)), self.h)
        return v.value

    def streamer_steps(self, parts: Particles, grid: DeviceGrid, n_pos: torch.Tensor, n_neg: torch.Tensor,
                       phi: torch.Tensor, dt: float, n_steps: int, seed: int, step0: int = 0, adaptive: bool = True,
                       dt_max: float | None = None, mu: dict | None = None, cfl: float = 0.5,
                       growth_max: float = 1.2, mg_tol: float = 1e-8, mg_max_cycles: int = 30,
                       E_out: torch.Tensor | None = None, check: bool = True, photo: dict | None = None):
        """Self-consistent steps (field from the densities before every step,
        ions from the step's events, Sec. 2.1.4 time step; photo: eta, k1, k2,
        w_photon of the photoionization after each step, Sec. 2.4).  Returns
        (rc, next dt, dt per step, stats)."""
        mu = mu or {"EN_lo": 1.0, "EN_hi": 10.0, "muN": np.array([0.0])}
        muN = np.ascontiguousarray(mu["muN"], dtype=np.float64)
        po = _photo_opts(photo) if photo is not None else None
        o = B.pcmcc_sc_opts(1 if adaptive else 0, float(dt_max if dt_max is not None else dt), float(cfl),
                            float(growth_max), int(muN.size), float(mu.get("EN_lo", 1.0)), float(mu.get("EN_hi", 10.0)),
                            muN.ctypes.data_as(C.c_void_p), float(mg_tol), int(mg_max_cycles),
                            C.pointer(po) if po is not None else None)
        d = C.c_double(dt)
        hist = np.zeros(max(n_steps, 1), dtype=np.float64)
        st = B.pcmcc_stats()
        ps, gs = parts.struct(), grid.struct()
        rc = B.lib().pcmcc_streamer_steps(self.h, C.byref(ps), C.byref(gs), n_pos.data_ptr(), n_neg.data_ptr(),
                                          phi.data_ptr(), C.c_void_p(E_out.data_ptr() if E_out is not None else 0),
                                          C.byref(o), int(n_steps), int(seed), int(step0), C.byref(d),
                                          hist.ctypes.data_as(C.c_void_p), C.byref(st))
        if check:
            B.check(rc, self.h)
        sd = st.as_dict()
        return rc, d.value, hist[:sd["steps_done"]], sd

    def photoionize(self, grid: DeviceGrid, ev: dict, photo: dict, seed: int, step: int, parts: Particles,
                    n_pos: torch.Tensor | None = None):
        """Photoelectrons of the ionization events ev (float32 device tensors
        x, y, z, w) appended to parts, their charge to n_pos (Sec. 2.4).
        Returns (photons emitted, photoelectrons appended)."""
        for k in ("x", "y", "z", "w"):
            assert ev[k].dtype == torch.float32 and ev[k].is_contiguous() and ev[k].numel() == ev["x"].numel()
        if n_pos is not None:
            assert n_pos.dtype == torch.int64 and n_pos.is_contiguous() and n_pos.numel() == grid.nx * grid.ny * grid.nz
        po = _photo_opts(photo)
        ph, ab = C.c_int64(0), C.c_int64(0)
        gs, ps = grid.struct(), parts.struct()
        B.check(B.lib().pcmcc_photoionize(self.h, C.byref(gs), ev["x"].data_ptr(), ev["y"].data_ptr(),
                                          ev["z"].data_ptr(), ev["w"].data_ptr(), int(ev["x"].numel()), C.byref(po),
                                          int(seed), int(step), C.byref(ps),
                                          C.c_void_p(n_pos.data_ptr() if n_pos is not None else 0), C.byref(ph),
                                          C.byref(ab)), self.h)
        return ph.value, ab.value

    def fluid_steps(self, grid: DeviceGrid, n_e: torch.Tensor, n_pos: torch.Tensor, n_neg: torch.Tensor,
                    phi: torch.Tensor, table: dict, dt_max: float, n_steps: int, mg_tol: float = 1e-8,
                    mg_max_cycles: int = 30, E_out: torch.Tensor | None = None, check: bool = True):
        """Fluid steps (Sec. 2.2) on float64 densities [nz][ny][nx] (in place);
        table: EN_lo, EN_hi and muN, DN, alphaN, etaN arrays on log-spaced
        E/N nodes.  Returns (rc, dt per step, stats)."""
        for t in (n_e, n_pos, n_neg, phi):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == grid.nx * grid.ny * grid.nz
        arrs = [np.ascontiguousarray(table[k], dtype=np.float64) for k in ("muN", "DN", "alphaN", "etaN")]
        tb = B.pcmcc_fluid_table(int(arrs[0].size), float(table["EN_lo"]), float(table["EN_hi"]),
                                 *[a.ctypes.data_as(C.c_void_p) for a in arrs])
        hist = np.zeros(max(n_steps, 1), dtype=np.float64)
        st = B.pcmcc_stats()
        gs = grid.struct()
        rc = B.lib().pcmcc_fluid_steps(self.h, C.byref(gs), n_e.data_ptr(), n_pos.data_ptr(), n_neg.data_ptr(),
                                       phi.data_ptr(), C.byref(tb), float(dt_max), float(mg_tol), int(mg_max_cycles),
                                       int(n_steps), hist.ctypes.data_as(C.c_void_p),
                                       C.c_void_p(E_out.data_ptr() if E_out is not None else 0), C.byref(st))
        if check:
            B.check(rc, self.h)
        sd = st.as_dict()
        return rc, hist[:sd["steps_done"]], sd

    def philox4x32_10(self, ctr: torch.Tensor, seed: int) -> torch.Tensor:
        assert ctr.dtype == torch.int32 and ctr.is_contiguous() and ctr.shape[-1] == 4
        out = torch.empty_like(ctr)
        B.check(B.lib().pcmcc_philox4x32_10(self.h, ctr.shape[0], ctr.data_ptr(), int(seed), out.data_ptr()),
                self.h)
        return out

    def tables_lookup(self, eps: torch.Tensor, n_proc: int, s_ub: torch.Tensor | None = None):
        n = eps.numel()
        cum = torch.empty((n, n_proc), dtype=torch.float32, device=eps.device)
        maj = torch.empty(n, dtype=torch.float32, device=eps.device) if s_ub is not None else None
        B.check(B.lib().pcmcc_tables_lookup(self.h, n, eps.data_ptr(), cum.data_ptr(),
                                            s_ub.data_ptr() if s_ub is not None else None,
                                            maj.data_ptr() if maj is not None else None), self.h)
        return cum, maj


def swarm_batch(ctx: Context, EN_Td, n0, dt: float, n_steps: int, seed: int, sample_every: int = 10,
                window_start_s: float = 0.0, n_batches: int = 10, cap_factor: int = 8,
                population_control: bool = True, block: int = 0, blocks_per_cu: int = 0, autotune: bool = False,
                tune_cache: str | None = None, raw: bool = False, check: bool = True, refill_min: int = 0,
                chunk: int = 0):
    """Batched uniform-field swarms (forwards to pcmcc_swarm_batch).

    Returns (rc, values[S, 14], errors[S, 14], stats[, moments[S, J, 14], counters[S, J, 4]])."""
    EN = np.ascontiguousarray(EN_Td, dtype=np.float64)
    n0 = np.ascontiguousarray(n0, dtype=np.int32)
    S = EN.size
    J = n_steps // sample_every
    opts = B.pcmcc_swarm_opts(int(sample_every), float(window_start_s), int(n_batches), int(cap_factor),
                              1 if population_control else 0, int(block), int(blocks_per_cu), 1 if autotune else 0,
                              tune_cache.encode() if tune_cache else None, int(refill_min), int(chunk))
    res = (B.pcmcc_swarm_result * S)()
    st = B.pcmcc_stats()
    mom = np.zeros((S, J, B.SWARM_NMOM)) if raw else None
    cnt = np.zeros((S, J, 4), dtype=np.int64) if raw else None
    rc = B.lib().pcmcc_swarm_batch(ctx.h, S, EN.ctypes.data_as(C.c_void_p), n0.ctypes.data_as(C.c_void_p),
                                   float(dt), int(n_steps), int(seed), C.byref(opts), res,
                                   mom.ctypes.data_as(C.c_void_p) if raw else None,
                                   cnt.ctypes.data_as(C.c_void_p) if raw else None, C.byref(st))
    if check:
        B.check(rc, ctx.h)
    vals = np.array([list(r.value) for r in res])
    errs = np.array([list(r.error) for r in res])
    out = (rc, vals, errs, st.as_dict())
    return out + ((mom, cnt) if raw else ())
