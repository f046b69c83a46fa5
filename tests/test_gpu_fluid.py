"""GPU parity of the fluid step (arXiv:2110.14494 Sec. 2.2) against the oracle.

The step is deterministic double-precision arithmetic; the GPU solves
Poisson's equation by multigrid (relative residual 1e-12) where the oracle
solves the discrete system exactly, and both round the field to single
precision, so densities are compared to 1e-7 of their largest value and the
time steps to 1e-9.
"""
import numpy as np
import pytest
import torch

from oracle import fluid as FL
from paper_2110_14494_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_14494_amd import pic as P
    return P


def _table():
    # transport data varying with E/N over 10-1000 Td (mobility falling,
    # diffusion and ionization rising, attachment falling)
    EN = 10.0 * 100.0 ** (np.arange(64) / 63)
    x = np.log(EN / 10.0) / np.log(100.0)
    return {"EN_lo": 10.0, "EN_hi": 1000.0, "muN": 4e24 * (1 - 0.6 * x), "DN": 1.5e25 * (1 + 2 * x),
            "alphaN": 1e-19 * x ** 3, "etaN": 5e-22 * (1 - x) ** 2}


@pytest.mark.parametrize("shape,dx,steps", [((16, 16, 16), 5e-5, 6), ((20, 12, 24), 4e-5, 4)])
def test_fluid_steps_match_oracle(pic, shape, dx, steps):
    nz, ny, nx = shape
    sp = W.electron_species()
    gas_N = sp["gas_N"]
    zc = (np.arange(nz) + 0.5) * dx - 0.6 * nz * dx
    yc = (np.arange(ny) + 0.5) * dx - 0.5 * ny * dx
    xc = (np.arange(nx) + 0.5) * dx - 0.45 * nx * dx
    z, y, x = np.meshgrid(zc, yc, xc, indexing="ij")
    blob = 5e19 * np.exp(-(x * x + y * y + z * z) / (2 * (2.5 * dx) ** 2))
    grid = {"E": np.zeros(shape + (4,), np.float32), "x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}
    grid["E"][..., 2] = 4e6
    grid["E"][..., 0] = 1e5
    tab = _table()
    ne_o, np_o, nn_o, info = FL.fluid_run(grid, blob, blob, np.zeros(shape), tab, gas_N, steps, 5e-12)
    ctx = pic.Context(0)
    ctx.init_species(sp)
    dg = pic.DeviceGrid(grid)
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (blob, blob.copy(), np.zeros(shape))]
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    E = torch.empty(shape + (4,), dtype=torch.float32, device="cuda")
    print(f"[gpu] fluid {shape} steps={steps}", flush=True)
    rc, hist, st = ctx.fluid_steps(dg, *t, phi, tab, 5e-12, steps, mg_tol=1e-12, mg_max_cycles=60, E_out=E,
                                   check=False)
    ne, npo, nne = (a.cpu().numpy() for a in t)
    Eg = E.cpu().numpy()
    ctx.close()
    assert rc == 0 and st["steps_done"] == steps
    print("[gpu] dt", hist, info["dt"], flush=True)
    assert np.allclose(hist, info["dt"], rtol=1e-9, atol=0)
    assert min(info["dt"]) < 5e-12  # a limit other than dt_max was active
    for g, o in ((ne, ne_o), (npo, np_o), (nne, nn_o)):
        assert np.max(np.abs(g - o)) <= 1e-7 * np.max(np.abs(o)), np.max(np.abs(g - o)) / np.max(np.abs(o))
    assert np.max(np.abs(Eg[..., :3] - info["E"])) <= 1e-6 * np.max(np.abs(info["E"]))


def test_fluid_streamer_grid_one_step(pic):
    # The fluid leg's full size: the 256^3 streamer grid (39 um cells, tip
    # field), the neutral Gaussian seed at the tip (peak 5.8e17 m^-3, sigma
    # 300 um), one Heun step against the oracle, with the same bars.
    cfg = W.streamer_config(n=2 ** 10)
    grid = cfg["grid"]
    E0 = np.asarray(grid["E"])
    nz, ny, nx = E0.shape[:3]
    dx = grid["dx"]
    c = [(np.arange(m) + 0.5) * dx for m in (nz, ny, nx)]
    tip = (8e-3, 5e-3, 5e-3)
    r2 = ((c[0] - tip[0]) ** 2)[:, None, None] + ((c[1] - tip[1]) ** 2)[None, :, None] + \
        ((c[2] - tip[2]) ** 2)[None, None, :]
    seed = 5.8e17 * np.exp(-r2 / (2 * 300e-6 ** 2))
    sp = W.electron_species()
    tab = _table()
    print(f"[gpu] fluid streamer grid {nx}^3, oracle step", flush=True)
    ne_o, np_o, nn_o, info = FL.fluid_run(grid, seed, seed, np.zeros_like(seed), tab, sp["gas_N"], 1, 2e-11)
    ctx = pic.Context(0)
    ctx.init_species(sp)
    dg = pic.DeviceGrid(grid)
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (seed, seed.copy(), np.zeros_like(seed))]
    phi = torch.zeros(seed.shape, dtype=torch.float64, device="cuda")
    E = torch.empty(seed.shape + (4,), dtype=torch.float32, device="cuda")
    print("[gpu] fluid streamer grid, GPU step", flush=True)
    rc, hist, st = ctx.fluid_steps(dg, *t, phi, tab, 2e-11, 1, mg_tol=1e-12, mg_max_cycles=80, E_out=E, check=False)
    ne, npo, nne = (a.cpu().numpy() for a in t)
    Eg = E.cpu().numpy()
    ctx.close()
    assert rc == 0 and st["steps_done"] == 1
    assert np.allclose(hist, info["dt"], rtol=1e-9, atol=0)
    for g, o in ((ne, ne_o), (npo, np_o), (nne, nn_o)):
        assert np.max(np.abs(g - o)) <= 1e-7 * np.max(np.abs(o)), np.max(np.abs(g - o)) / np.max(np.abs(o))
    assert np.max(np.abs(Eg[..., :3] - info["E"])) <= 1e-6 * np.max(np.abs(info["E"]))
