"""GPU parity of the self-consistent step (arXiv:2110.14494 Sec. 2.5 Poisson's
equation and E = -grad phi, Sec. 2.3 boundary conditions, Sec. 2.1.4 time
step) against the oracle.

Bars: the multigrid potential within 1e-9 of the oracle's exact discrete
solution (relative to its largest value) at a residual tolerance of 1e-12;
the field from a given potential bit for bit; the 90 % speed quantile bit for
bit; a weakly coupled run within the step tests' bars (state within 1e-5,
flips below 1e-4 of the flight segments), the same ion charge up to the
flipped lineages and an exact charge balance; a strongly coupled adaptive run
as an ensemble (time steps to 1e-4, count and charges to 1 %, mean energy
to 2 %, field to 5 %).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import field as F
from paper_2110_14494_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_14494_amd import pic as P
    return P


def _grid(nx, ny, nz, dx, Ez=0.0):
    E = np.zeros((nz, ny, nx, 4), np.float32)
    E[..., 2] = Ez
    return {"E": E, "x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}


def _densities(shape, seed):
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 2 ** 40, size=shape, dtype=np.int64)
    blob = np.zeros(shape, np.int64)
    nz, ny, nx = shape
    blob[nz // 3:nz // 2, ny // 4:ny // 2, nx // 3:2 * nx // 3] = 2 ** 44
    n_pos = base + blob
    n_e = rng.integers(0, 2 ** 40, size=shape, dtype=np.int64)
    n_neg = rng.integers(0, 2 ** 36, size=shape, dtype=np.int64)
    return n_pos, n_e, n_neg


@pytest.mark.parametrize("shape,dx", [((16, 16, 16), 5e-5), ((24, 40, 32), 2e-5), ((64, 64, 64), 4e-5)])
def test_potential_matches_exact_discrete_solution(pic, shape, dx):
    nz, ny, nx = shape
    grid = _grid(nx, ny, nz, dx)
    n_pos, n_e, n_neg = _densities(shape, 7)
    ref = F.poisson(F.charge_density(n_pos, n_e, n_neg, dx), dx)
    ctx = pic.Context(0)
    dg = pic.DeviceGrid(grid)
    t = [torch.from_numpy(a).cuda() for a in (n_pos, n_e, n_neg)]
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    print(f"[gpu] potential {shape}", flush=True)
    cyc, rel = ctx.solve_potential(dg, *t, phi, tol=1e-12, max_cycles=60)
    got = phi.cpu().numpy()
    # a warm start from the solution converges at once
    cyc2, rel2 = ctx.solve_potential(dg, *t, phi, tol=1e-12, max_cycles=60)
    ctx.close()
    print(f"[gpu] cycles {cyc} rel {rel:.2e}; warm {cyc2}", flush=True)
    assert rel <= 1e-12 and cyc < 40 and cyc2 <= 2
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_field_from_potential_bit_exact(pic):
    nz, ny, nx, dx = 12, 20, 16, 3e-5
    grid = _grid(nx, ny, nz, dx, Ez=1.5e6)
    grid["E"][..., 0] = np.random.default_rng(1).normal(0, 1e5, (nz, ny, nx)).astype(np.float32)
    phi = np.random.default_rng(2).normal(0, 10.0, (nz, ny, nx))
    ref = F.field(phi, grid["E"], dx)
    ctx = pic.Context(0)
    dg = pic.DeviceGrid(grid)
    E = ctx.field_from_potential(dg, torch.from_numpy(phi).cuda()).cpu().numpy()
    ctx.close()
    assert np.array_equal(E[..., :3], ref) and np.all(E[..., 3] == 0)


@pytest.mark.parametrize("n", [1, 2, 10, 11, 1000, 1_048_579])
def test_speed_quantile_exact(pic, n):
    rng = np.random.default_rng(n + 5)
    v = rng.normal(0, 2e5, (3, n)).astype(np.float32)
    if n > 8:
        v[:, : n // 4] = v[:, :1]  # a quarter of ties
    parts = {"x": np.zeros(n, np.float32), "y": np.zeros(n, np.float32), "z": np.zeros(n, np.float32),
             "vx": v[0], "vy": v[1], "vz": v[2], "w": np.ones(n, np.float32), "id": np.arange(n, dtype=np.uint64)}
    ctx = pic.Context(0)
    dp = pic.Particles.from_numpy(parts, n)
    got = ctx.speed_quantile(dp)
    ctx.close()
    assert got == F.v90(*v)


def qsum(a):
    """Exact sum of fixed-point charge counts (an int64 sum overflows at
    thousands of electrons of weight 1e6, each 1e6 * 2^32)."""
    return int(np.asarray(a).astype(object).sum())


def _coupled_case(n=3000, w=1e4):
    cfg = W.plain_swarm_config(n=n)
    cfg["grid"] = W.uniform_grid(16, 80e-6, (0.0, 0.0, 1.0e7))
    parts = W.uniform_box_particles(n, 0.45e-3, 0.85e-3, 3e5, seed=8)
    parts["w"][:] = w
    return cfg, parts


def _run_pair(pic, w, dt_max, steps, adaptive, neutral=True):
    cfg, parts = _coupled_case(w=w)
    grid = cfg["grid"]
    mu = {"EN_lo": 10.0, "EN_hi": 1000.0, "muN": np.array([4e24, 2e24, 1e24, 0.8e24])}
    seed = 3
    n = parts["x"].size
    n_pos0 = oracle.deposit(parts["x"], parts["y"], parts["z"], parts["w"], grid)  # neutral seed
    if not neutral:
        n_pos0[:] = 0
    n_pos_o, n_neg_o = n_pos0.copy(), np.zeros_like(n_pos0)
    orc_rc, o, info = F.streamer_run(cfg["species"], cfg["tables"], grid, parts, n_pos_o, n_neg_o, 1e-12, steps,
                                     seed, dt_max=dt_max, mu=mu, capacity=16 * n, adaptive=adaptive)
    assert orc_rc == 0
    ctx = pic.Context(0)
    ctx.setup(cfg["species"], cfg["tables"])
    dp = pic.Particles.from_numpy(parts, 16 * n)
    dg = pic.DeviceGrid(grid)
    n_pos = torch.from_numpy(n_pos0.copy()).cuda()
    n_neg = torch.zeros_like(n_pos)
    phi = torch.zeros(n_pos.shape, dtype=torch.float64, device="cuda")
    E = torch.empty((16, 16, 16, 4), dtype=torch.float32, device="cuda")
    print(f"[gpu] coupled steps w={w} adaptive={adaptive}", flush=True)
    rc, dt_next, hist, st = ctx.streamer_steps(dp, dg, n_pos, n_neg, phi, 1e-12, steps, seed, adaptive=adaptive,
                                               dt_max=dt_max, mu=mu, mg_tol=1e-12, mg_max_cycles=60, E_out=E,
                                               check=False)
    g = dp.to_numpy()
    gpu = {"parts": g, "n_pos": n_pos.cpu().numpy(), "n_neg": n_neg.cpu().numpy(), "E": E.cpu().numpy()[..., :3],
           "dt": hist, "next_dt": dt_next, "stats": st}
    ctx.close()
    assert rc == 0 and st["steps_done"] == steps
    print("[gpu] dt", hist, info["dt"], dt_next, info["next_dt"], flush=True)
    return grid, gpu, (o, n_pos_o, n_neg_o, info)


def test_coupled_steps_match_oracle(pic):
    # An electron cloud without ions, weights of 100: the space-charge field
    # is ~5e-4 of the applied field (a wrong sign or scale of the coupling
    # shows in every electron), while one lineage that decides differently
    # moves its neighbours' field by ~2e-6 only, so the step tests'
    # per-electron bar holds.
    from test_gpu_pic import compare
    w, steps = 100.0, 6
    grid, gpu, (o, n_pos_o, n_neg_o, info) = _run_pair(pic, w, 2e-12, steps, adaptive=False, neutral=False)
    g = gpu["parts"]
    assert np.array_equal(gpu["dt"], info["dt"])
    res = compare(g, {k: np.asarray(v) for k, v in o.items()}, grid["dx"])
    print("[gpu] parity", res, flush=True)
    assert res["flips"] <= max(1e-4 * gpu["stats"]["trials"], 2), res
    # the same ion charge created up to the flipped lineages, exact balance
    tol = (res["flips"] + 2) * int(w) * 2 ** 32
    assert abs(qsum(gpu["n_pos"]) - qsum(n_pos_o)) <= tol
    assert abs(qsum(gpu["n_neg"]) - qsum(n_neg_o)) <= tol
    n_e_g = oracle.deposit(g["x"], g["y"], g["z"], g["w"], grid)
    n_e_0 = oracle.deposit(*(np.asarray(_coupled_case(w=w)[1][k]) for k in ("x", "y", "z", "w")), grid)
    # ions created = electrons gained (no electron left the box)
    assert qsum(gpu["n_pos"]) - qsum(gpu["n_neg"]) == qsum(n_e_g) - qsum(n_e_0)
    scale = np.max(np.abs(info["E"]))
    assert np.max(np.abs(gpu["E"] - info["E"])) <= 1e-5 * scale
    # the space charge matters at this weight: the field is not the applied one
    assert np.max(np.abs(info["E"] - np.asarray(grid["E"])[..., :3])) > 1e-4 * scale


def test_coupled_adaptive_steps_match_oracle_in_ensemble(pic):
    # Weights of 1e6 with the adaptive step: the CFL limit (second step), the
    # 20 % growth limit and the dielectric relaxation limit take turns.  The
    # run is strongly coupled (one lineage deciding differently moves its
    # neighbours' field by ~1e-2 and the growth limit by ~1e-6), so electrons
    # are compared as an ensemble: time steps, count, charge, mean energy,
    # field.
    w, steps = 1e6, 8
    grid, gpu, (o, n_pos_o, n_neg_o, info) = _run_pair(pic, w, 1e-10, steps, adaptive=True)
    g = gpu["parts"]
    # The growth limit divides by ln(N_new / N_old) ~ ln 1.2, so each electron
    # that a flipped lineage adds or removes moves the next step by about
    # 1 / (N ln 1.2) ~ 1.4e-3 at N ~ 4000: the bar allows a few such electrons.
    assert np.allclose(gpu["dt"], info["dt"], rtol=1e-2, atol=0)
    assert math.isclose(gpu["next_dt"], info["next_dt"], rel_tol=1e-2)
    assert min(info["dt"][1:]) < 0.05 * 1e-10  # the limits were active
    assert abs(g["x"].size / o["x"].size - 1) < 0.01
    for a, b in ((gpu["n_pos"], n_pos_o), (gpu["n_neg"], n_neg_o)):
        assert abs(qsum(a) - qsum(b)) <= 0.01 * max(qsum(b), int(w) * 2 ** 32)
    ke = lambda d: float(np.mean(np.asarray(d["vx"], np.float64) ** 2 + np.asarray(d["vy"], np.float64) ** 2 +
                                 np.asarray(d["vz"], np.float64) ** 2))
    assert abs(ke(g) / ke(o) - 1) < 0.02
    scale = np.max(np.abs(info["E"]))
    assert np.max(np.abs(gpu["E"] - info["E"])) <= 0.05 * scale
    n_e_g = oracle.deposit(g["x"], g["y"], g["z"], g["w"], grid)
    assert qsum(gpu["n_pos"]) - qsum(n_e_g) - qsum(gpu["n_neg"]) == 0


def test_error_paths(pic):
    # a grid that does not coarsen to a small enough level, missing species,
    # invalid options: errors, not faults
    from paper_2110_14494_amd import _binding as B
    ctx = pic.Context(0)
    g = _grid(65, 65, 65, 1e-5)
    dg = pic.DeviceGrid(g)
    z = torch.zeros((65, 65, 65), dtype=torch.int64, device="cuda")
    phi = torch.zeros((65, 65, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PcmccError) as e:
        ctx.solve_potential(dg, z, z, z, phi)
    assert e.value.code == B.PCMCC_EINVAL
    dg8 = pic.DeviceGrid(_grid(8, 8, 8, 1e-5))
    d8 = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    tab = {"EN_lo": 10.0, "EN_hi": 1000.0, "muN": np.ones(4), "DN": np.ones(4), "alphaN": np.zeros(4),
           "etaN": np.zeros(4)}
    rc, _, _ = ctx.fluid_steps(dg8, d8, d8.clone(), d8.clone(), d8.clone(), tab, 1e-12, 1, check=False)
    assert rc == B.PCMCC_ESTATE  # no species yet: the gas density is unknown
    ctx.init_species(W.electron_species())
    bad = dict(tab, EN_hi=5.0)
    rc, _, _ = ctx.fluid_steps(dg8, d8, d8.clone(), d8.clone(), d8.clone(), bad, 1e-12, 1, check=False)
    assert rc == B.PCMCC_EINVAL
    rc, _, _ = ctx.fluid_steps(dg8, d8, d8.clone(), d8.clone(), d8.clone(), tab, -1.0, 1, check=False)
    assert rc == B.PCMCC_EINVAL
    cfg, parts = _coupled_case(n=100)
    ctx.setup(cfg["species"], cfg["tables"])
    dp = pic.Particles.from_numpy(parts, 1000)
    dg16 = pic.DeviceGrid(cfg["grid"])
    n16 = torch.zeros((16, 16, 16), dtype=torch.int64, device="cuda")
    p16 = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    rc, _, _, _ = ctx.streamer_steps(dp, dg16, n16, n16.clone(), p16, 1e-12, 1, 0, growth_max=0.5, check=False)
    assert rc == B.PCMCC_EINVAL
    rc, _, _, _ = ctx.streamer_steps(dp, dg16, n16, n16.clone(), p16, -1e-12, 1, 0, check=False)
    assert rc == B.PCMCC_EINVAL
    assert dp.n == 100  # nothing moved
    ctx.close()


def test_streamer_full_size_two_coupled_steps(pic):
    # The self-consistent leg's full size: 2^24 electrons on the 256^3
    # streamer grid with the neutral seed, two steps in the space-charge
    # field against the oracle.  The first step's field is the applied one
    # (no net charge), the second sees the charge the first separated: a weak
    # coupling, so lineages are compared electron by electron with the step
    # tests' bars, plus the field, the ion charge and the exact balance.
    from test_gpu_pic import compare
    cfg = W.streamer_config()
    parts, grid = cfg["parts"], cfg["grid"]
    n = parts["x"].size
    n_pos0 = oracle.deposit(parts["x"], parts["y"], parts["z"], parts["w"], grid)
    n_pos_o, n_neg_o = n_pos0.copy(), np.zeros_like(n_pos0)
    print(f"[gpu] full-size coupled steps n={n}: oracle", flush=True)
    orc_rc, o, info = F.streamer_run(cfg["species"], cfg["tables"], grid, parts, n_pos_o, n_neg_o, cfg["dt"], 2,
                                     cfg["seed"], capacity=4 * n, adaptive=False)
    assert orc_rc == 0
    ctx = pic.Context(0)
    ctx.setup(cfg["species"], cfg["tables"])
    dp = pic.Particles.from_numpy(parts, 4 * n)
    dg = pic.DeviceGrid(grid)
    n_pos = torch.from_numpy(n_pos0.copy()).cuda()
    n_neg = torch.zeros_like(n_pos)
    phi = torch.zeros(n_pos.shape, dtype=torch.float64, device="cuda")
    E = torch.empty(tuple(n_pos.shape) + (4,), dtype=torch.float32, device="cuda")
    print("[gpu] full-size coupled steps: GPU", flush=True)
    rc, _, hist, st = ctx.streamer_steps(dp, dg, n_pos, n_neg, phi, cfg["dt"], 2, cfg["seed"], adaptive=False,
                                         mg_tol=1e-12, mg_max_cycles=80, E_out=E, check=False)
    g = dp.to_numpy()
    gp, gn, Eg = n_pos.cpu().numpy(), n_neg.cpu().numpy(), E.cpu().numpy()[..., :3]
    ctx.close()
    assert rc == 0 and st["steps_done"] == 2 and st["lost"] == 0
    res = compare(g, {k: np.asarray(v) for k, v in o.items()}, grid["dx"])
    print("[gpu] parity", res, flush=True)
    assert res["flips"] <= max(1e-4 * st["trials"], 2), res
    assert res["matched"] >= 0.999 * o["id"].size
    tol = (res["flips"] + 2) * int(np.max(parts["w"])) * 2 ** 32
    assert abs(qsum(gp) - qsum(n_pos_o)) <= tol
    assert abs(qsum(gn) - qsum(n_neg_o)) <= tol
    n_e = oracle.deposit(g["x"], g["y"], g["z"], g["w"], grid)
    assert qsum(gp) - qsum(gn) == qsum(n_e)  # neutral: ions = electrons, exactly
    scale = np.max(np.abs(info["E"]))
    assert np.max(np.abs(Eg - info["E"])) <= 1e-5 * scale
    # the second step's field is not the applied one
    assert np.max(np.abs(info["E"] - np.asarray(grid["E"])[..., :3])) > 1e-6 * scale
