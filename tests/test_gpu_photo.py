"""GPU parity of the discrete photoionization (arXiv:2110.14494 Sec. 2.4)
against the oracle.

Bars: the same photon count and the same photoelectrons by id (positions
within 2 single-precision ulps: both sides compute the absorption point in
double precision, E1 and the sines may differ in the last bit; weights exact),
photons absorbed right at a box face allowed to differ (at most 1e-4 of them);
the ion charge added to n_pos bit-exact against the oracle's deposit of the
GPU's photoelectrons; the particles present before the call untouched.  In
the self-consistent steps: the photon count of the Bernoulli yield within 5
sigma of eta times the ionizations, and the exact charge balance (ions created
= electrons gained) with the photo-ions included.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import photo as P

pytestmark = pytest.mark.gpu

K = [(5.25e3, 3.0e5), (2.0e4, 1.0e6)]


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_14494_amd import pic as P_
    return P_


def _grid(n=64, dx=1e-5):
    E = np.zeros((n, n, n, 4), np.float32)
    return {"E": E, "x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}, n


def _events(n, seed, box):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.05 * box, 0.95 * box, size=(n, 3)).astype(np.float32)
    w = rng.uniform(1.0, 2000.0, n).astype(np.float32)
    return {"x": pos[:, 0].copy(), "y": pos[:, 1].copy(), "z": pos[:, 2].copy(), "w": w}


def _ulps(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return np.abs(a.astype(np.float64) - b.astype(np.float64)) / np.spacing(np.maximum(np.abs(a), np.abs(b)))


@pytest.mark.parametrize("k", K)
@pytest.mark.parametrize("eta,w_photon", [(0.0028846, 1.0), (0.3, 0.0)])
def test_photoionize_matches_oracle(pic, k, eta, w_photon):
    grid, nc = _grid()
    n_ev, n0 = 40_000, 1000
    ev = _events(n_ev, 3, nc * grid["dx"])
    seed, step = 0x1234_5678_9ABC, 17
    o = P.photoionize(ev["x"], ev["y"], ev["z"], ev["w"], grid, eta, k[0], k[1], w_photon, seed, step, nc, nc, nc)
    ctx = pic.Context(0)
    dg = pic.DeviceGrid(grid)
    rng = np.random.default_rng(5)
    pre = {c: rng.uniform(1e-4, 5e-4, n0).astype(np.float32) for c in ("x", "y", "z", "vx", "vy", "vz", "w")}
    pre["id"] = rng.integers(0, 2 ** 63, n0, dtype=np.uint64)
    parts = pic.Particles.from_numpy(pre, n0 + o["photons"] + 10)
    n_pos = dg.zeros_rho()
    dev = {c: torch.from_numpy(ev[c]).cuda() for c in ev}
    print(f"[gpu] photoionize k={k} eta={eta} w_photon={w_photon}: oracle {o['photons']} photons, "
          f"{o['absorbed']} absorbed", flush=True)
    ph, ab = ctx.photoionize(dg, dev, {"eta": eta, "k1": k[0], "k2": k[1], "w_photon": w_photon}, seed, step, parts,
                             n_pos)
    g = parts.to_numpy()
    rho = n_pos.cpu().numpy()
    ctx.close()
    assert ph == o["photons"] and o["photons"] > 1000
    assert g["x"].size == n0 + ab
    for c in pre:
        assert np.array_equal(g[c][:n0], pre[c])
    new = {c: g[c][n0:] for c in g}
    common, ig, io = np.intersect1d(new["id"], o["id"], return_indices=True)
    assert len(new["id"]) - len(common) <= max(1, 1e-4 * ab) and len(o["id"]) - len(common) <= max(1, 1e-4 * ab)
    for c in ("x", "y", "z"):
        assert np.max(_ulps(new[c][ig], o[c][io])) <= 2.0, c
    assert np.array_equal(new["w"][ig], o["w"][io])
    assert np.all(new["vx"] == 0) and np.all(new["vy"] == 0) and np.all(new["vz"] == 0)
    assert np.array_equal(rho, oracle.deposit(new["x"], new["y"], new["z"], new["w"], grid))


def test_photoionize_many_photons_per_event(pic):
    # lambda up to 200 photons per event (weights up to 2000, single photons):
    # the per-event photon index j runs far beyond the first draw words
    grid, nc = _grid(32, 2e-5)
    ev = _events(2000, 9, nc * grid["dx"])
    k1, k2 = 2.0e4, 1.0e6
    o = P.photoionize(ev["x"], ev["y"], ev["z"], ev["w"], grid, 0.1, k1, k2, 1.0, 5, 2, nc, nc, nc)
    ctx = pic.Context(0)
    dg = pic.DeviceGrid(grid)
    parts = pic.Particles(o["photons"] + 1)
    n_pos = dg.zeros_rho()
    dev = {c: torch.from_numpy(ev[c]).cuda() for c in ev}
    print(f"[gpu] photoionize many photons: oracle {o['photons']}", flush=True)
    ph, ab = ctx.photoionize(dg, dev, {"eta": 0.1, "k1": k1, "k2": k2, "w_photon": 1.0}, 5, 2, parts, n_pos)
    g = parts.to_numpy()
    rho = n_pos.cpu().numpy()
    ctx.close()
    assert ph == o["photons"] and ph > 150_000
    common, ig, io = np.intersect1d(g["id"], o["id"], return_indices=True)
    assert ab - len(common) <= max(1, 1e-4 * ab) and o["absorbed"] - len(common) <= max(1, 1e-4 * ab)
    for c in ("x", "y", "z"):
        assert np.max(_ulps(g[c][ig], o[c][io])) <= 2.0, c
    assert np.all(g["w"] == 1.0)
    assert np.array_equal(rho, oracle.deposit(g["x"], g["y"], g["z"], g["w"], grid))


def test_photoionize_streamer_scale(pic):
    # The self-consistent streamer stage's scale: 1e6 ionization events around
    # the tip (N(tip, 300 um)) on the 256^3 grid of 10 mm, the paper's yield
    # (xi 0.075, p_q 40 mbar at 1 bar) with photons of the event's weight and
    # the absorption constants of air: every photon compared with the oracle.
    from paper_2110_14494_amd import workloads as W
    cfg = W.streamer_config(n=2 ** 10)
    grid = cfg["grid"]
    nz, ny, nx = np.asarray(grid["E"]).shape[:3]
    rng = np.random.default_rng(11)
    n_ev = 1_000_000
    tip = np.array([5e-3, 5e-3, 8e-3])
    pos = (tip + 300e-6 * rng.standard_normal((n_ev, 3))).astype(np.float32)
    ev = {"x": pos[:, 0].copy(), "y": pos[:, 1].copy(), "z": pos[:, 2].copy(),
          "w": rng.uniform(200.0, 2000.0, n_ev).astype(np.float32)}
    eta = 40.0 / 1040.0 * 0.075
    photo = {"eta": eta, "k1": 5.25e3, "k2": 3.0e5, "w_photon": 0.0}
    o = P.photoionize(ev["x"], ev["y"], ev["z"], ev["w"], grid, eta, 5.25e3, 3.0e5, 0.0, 77, 123, nx, ny, nz)
    ctx = pic.Context(0)
    dg = pic.DeviceGrid(grid)
    parts = pic.Particles(o["photons"] + 16)
    n_pos = dg.zeros_rho()
    dev = {c: torch.from_numpy(ev[c]).cuda() for c in ev}
    print(f"[gpu] photoionize streamer scale: oracle {o['photons']} photons", flush=True)
    ph, ab = ctx.photoionize(dg, dev, photo, 77, 123, parts, n_pos)
    g = parts.to_numpy()
    rho = n_pos.cpu().numpy()
    ctx.close()
    assert ph == o["photons"] and abs(ph - eta * n_ev) < 5 * math.sqrt(eta * n_ev)
    common, ig, io = np.intersect1d(g["id"], o["id"], return_indices=True)
    assert ab - len(common) <= 1 and o["absorbed"] - len(common) <= 1
    for c in ("x", "y", "z"):
        assert np.max(_ulps(g[c][ig], o[c][io])) <= 2.0, c
    assert np.array_equal(g["w"][ig], o["w"][io])
    assert np.array_equal(rho, oracle.deposit(g["x"], g["y"], g["z"], g["w"], grid))


def test_photoionize_capacity_empty_and_errors(pic):
    grid, nc = _grid(16, 4e-5)
    ev = _events(5000, 4, nc * grid["dx"])
    photo = {"eta": 0.5, "k1": 5.25e3, "k2": 3.0e5, "w_photon": 0.0}
    ctx = pic.Context(0)
    dg = pic.DeviceGrid(grid)
    dev = {c: torch.from_numpy(ev[c]).cuda() for c in ev}
    pre = {c: np.full(10, 1e-4, np.float32) for c in ("x", "y", "z", "vx", "vy", "vz", "w")}
    pre["id"] = np.arange(10, dtype=np.uint64)
    print("[gpu] photoionize capacity", flush=True)
    parts = pic.Particles.from_numpy(pre, 100)  # room for 90 of about 2500 photons
    n_pos = dg.zeros_rho()
    with pytest.raises(pic.B.PcmccError) as e:
        ctx.photoionize(dg, dev, photo, 1, 0, parts, n_pos)
    assert e.value.code == pic.B.PCMCC_ECAPACITY
    assert parts.n == 10 and int(n_pos.abs().sum()) == 0
    empty = {c: dev[c][:0] for c in dev}
    assert ctx.photoionize(dg, empty, photo, 1, 0, parts, n_pos) == (0, 0)
    for bad in ({"eta": -1.0, "k1": 1.0, "k2": 2.0}, {"eta": 0.1, "k1": 2.0, "k2": 1.0},
                {"eta": 0.1, "k1": 0.0, "k2": 1.0}, {"eta": float("nan"), "k1": 1.0, "k2": 2.0}):
        with pytest.raises(pic.B.PcmccError) as e:
            ctx.photoionize(dg, dev, bad, 1, 0, parts, n_pos)
        assert e.value.code == pic.B.PCMCC_EINVAL
    # no n_pos: photoelectrons only
    big = pic.Particles.from_numpy(pre, 10_000)
    ph, ab = ctx.photoionize(dg, dev, photo, 1, 0, big, None)
    assert big.n == 10 + ab and 0 < ab <= ph
    # free slots exactly equal to the photons emitted: accepted
    exact = pic.Particles.from_numpy(pre, 10 + ph)
    ph2, ab2 = ctx.photoionize(dg, dev, photo, 1, 0, exact, None)
    assert (ph2, ab2) == (ph, ab) and exact.n == 10 + ab
    # one slot fewer: refused, nothing written
    short = pic.Particles.from_numpy(pre, 9 + ph)
    with pytest.raises(pic.B.PcmccError) as e:
        ctx.photoionize(dg, dev, photo, 1, 0, short, None)
    assert e.value.code == pic.B.PCMCC_ECAPACITY and short.n == 10
    ctx.close()


def test_streamer_steps_with_photoionization(pic):
    # absorption lengths of 20 um and 1 um: no photon reaches the box faces
    # (0.4 mm away), so no electron leaves and the charge balance is exact
    from test_gpu_field import _coupled_case
    cfg, parts = _coupled_case(w=100.0)
    grid = cfg["grid"]
    n = parts["x"].size
    eta = 0.5
    ctx = pic.Context(0)
    ctx.setup(cfg["species"], cfg["tables"])
    dp = pic.Particles.from_numpy(parts, 16 * n)
    dg = pic.DeviceGrid(grid)
    n_e0 = oracle.deposit(parts["x"], parts["y"], parts["z"], parts["w"], grid)
    n_pos = torch.zeros(n_e0.shape, dtype=torch.int64, device="cuda")
    n_neg = torch.zeros_like(n_pos)
    phi = torch.zeros(n_pos.shape, dtype=torch.float64, device="cuda")
    print("[gpu] streamer steps with photoionization", flush=True)
    rc, _, hist, st = ctx.streamer_steps(dp, dg, n_pos, n_neg, phi, 1e-12, 6, 3, adaptive=False, dt_max=2e-12,
                                         mg_tol=1e-10, mg_max_cycles=60,
                                         photo={"eta": eta, "k1": 5.0e4, "k2": 1.0e6, "w_photon": 0.0})
    g = dp.to_numpy()
    ctx.close()
    assert rc == 0 and st["steps_done"] == 6
    n_ion = st["ionization"]
    print(f"[gpu] ionizations {n_ion}, photons {st['photons']}, photoelectrons {st['photoelectrons']}", flush=True)
    assert n_ion > 50
    assert abs(st["photons"] - eta * n_ion) <= 5 * math.sqrt(n_ion * eta * (1 - eta))
    assert 0 < st["photoelectrons"] <= st["photons"] and st["photo_ms"] > 0
    assert st["lost"] == 0
    # every ion has its electron: ionization newborns and photoelectrons (no electron left the box)
    n_e = oracle.deposit(g["x"], g["y"], g["z"], g["w"], grid)
    assert int(n_pos.sum()) - int(n_neg.sum()) == int(n_e.sum()) - int(n_e0.sum())
