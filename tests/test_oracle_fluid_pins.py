"""Pins of the oracle's fluid step (arXiv:2110.14494 Sec. 2.2: drift-diffusion-
reaction equation, Koren-limited advection, central diffusion, Heun's method,
time-step limits).

Checks: the limiter's values, exact drift of a linear profile, the diffusion
operator against a separately written Neumann 7-point Laplacian with exact
mass conservation, exponential growth and its second-order convergence, each
time-step limit in closed form, and charge conservation of a coupled run.
"""
import math

import numpy as np
import pytest

from oracle import field as F
from oracle import fluid as FL

GAS_N = 2.45e25


def _tab(mu=3e24, D=1.5e25, alpha=0.0, eta=0.0):
    one = np.ones(4)
    return {"EN_lo": 10.0, "EN_hi": 1000.0, "muN": mu * one, "DN": D * one, "alphaN": alpha * one, "etaN": eta * one}


def test_koren_limiter_values():
    a = np.array([1.0, 1.0, 1.0, 1.0, 1.0, -2.0, 2.0, 0.0])
    b = np.array([-1.0, 0.25, 1.0, 4.0, 0.0, -2.0, 1.0, 3.0])
    # r = b / a: -1 -> 0; 0.25 -> 0.5; 1 -> 1; 4 -> 2; 0 -> 0; r = 1 with a < 0 -> a; r = 0.5 -> 2/3; a = 0 -> 0
    want = np.array([0.0, 0.5, 1.0, 2.0, 0.0, -2.0, 2.0 * (2.0 / 3.0), 0.0])
    assert np.allclose(FL.koren(a, b), want, rtol=0, atol=1e-15)


def test_drift_of_a_linear_profile_is_exact():
    nz, ny, nx, dx = 3, 4, 16, 1e-5
    x = (np.arange(nx) + 0.5) * dx
    n = np.broadcast_to(1e18 + 3e21 * x, (nz, ny, nx)).copy()
    E = np.zeros((nz, ny, nx, 3), np.float32)
    E[..., 0] = -2e6  # v = -mu E = +mu 2e6 along x
    tab = _tab(D=0.0)
    dne, dnp, dnn = FL.derivatives(n, E, dx, tab, GAS_N)
    v = 3e24 / GAS_N * 2e6
    inner = dne[:, :, 2:-2]
    assert np.allclose(inner, -v * 3e21, rtol=1e-9)
    assert np.all(dnp == 0) and np.all(dnn == 0)


def test_diffusion_matches_a_neumann_laplacian_and_conserves_mass():
    rng = np.random.default_rng(4)
    nz, ny, nx, dx = 6, 7, 9, 2e-5
    n = rng.uniform(0, 1e18, (nz, ny, nx))
    E = np.zeros((nz, ny, nx, 3), np.float32)
    D = 1.5e25 / GAS_N
    dne, _, _ = FL.derivatives(n, E, dx, _tab(), GAS_N)
    # Neumann 7-point Laplacian written as sums of neighbour differences
    lap = np.zeros_like(n)
    for ax in range(3):
        d = np.diff(n, axis=ax)  # n[i+1] - n[i] on interior faces
        pad = [(0, 0)] * 3
        pad[ax] = (1, 1)
        f = np.pad(d, pad)  # zero flux on boundary faces
        lap += np.diff(f, axis=ax)
    lap /= dx * dx
    assert np.allclose(dne, D * lap, rtol=1e-9, atol=1e-9 * np.abs(D * lap).max())
    assert abs(dne.sum()) <= 1e-9 * np.abs(dne).sum()


def _uniform_run(dt_max, steps, alpha=3e-20):
    shape = (4, 4, 4)
    grid = {"E": np.zeros(shape + (4,), np.float32), "x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": 1e-4}
    grid["E"][..., 2] = 5e6
    n0 = np.full(shape, 1e16)
    ne, npo, nne, info = FL.fluid_run(grid, n0, n0.copy(), np.zeros(shape), _tab(D=0.0, alpha=alpha), GAS_N, steps,
                                      dt_max)
    return ne, npo, nne, info


def test_uniform_growth_is_exponential_and_second_order():
    # neutral uniform plasma: the space charge stays zero, n grows as
    # exp(alpha mu |E| t); Heun's error falls four-fold when dt halves
    alpha = 3e-20  # alpha / N
    rate = alpha * GAS_N * (3e24 / GAS_N) * 5e6
    errs = []
    for dt, steps in ((1e-13, 10), (5e-14, 20)):  # rate dt = 0.045 and 0.0225
        ne, npo, nne, info = _uniform_run(dt, steps, alpha)
        assert all(d == dt for d in info["dt"])
        exact = 1e16 * math.exp(rate * dt * steps)
        assert np.allclose(ne, ne.flat[0], rtol=1e-12) and np.allclose(npo, ne, rtol=1e-12)
        errs.append(abs(ne.flat[0] / exact - 1))
    assert errs[0] < 1e-3 and 3.5 < errs[0] / errs[1] < 4.5, errs


def test_time_step_limits():
    shape, dx = (3, 3, 3), 1e-5
    E = np.zeros(shape + (3,), np.float32)
    n = np.zeros(shape)
    mu, D = 3e24 / GAS_N, 1.5e25 / GAS_N
    assert FL.time_step(n, E, dx, _tab(), GAS_N, 1.0) == pytest.approx(0.9 * 0.5 * dx * dx / (6 * D), rel=1e-12)
    E[1, 1, 1] = (1e6, -2e6, 3e6)
    want = 0.9 * 0.5 / (6 * D / dx ** 2 + mu * 6e6 / dx)
    assert FL.time_step(n, E, dx, _tab(), GAS_N, 1.0) == pytest.approx(want, rel=1e-12)
    n[0, 2, 1] = 1e21
    drt = F.EPS0 / (F.QE * 1e21 * mu)
    assert FL.time_step(n, np.zeros_like(E), dx, _tab(D=0.0), GAS_N, 1.0) == pytest.approx(0.9 * drt, rel=1e-12)
    assert FL.time_step(n, E, dx, _tab(), GAS_N, 1e-15) == 1e-15


def test_coupled_run_conserves_charge_away_from_the_boundary():
    nz = ny = nx = 16
    dx = 5e-5
    c = (np.arange(nx) + 0.5) * dx - 0.5 * nx * dx
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    blob = 1e18 * np.exp(-(x * x + y * y + z * z) / (2 * (5e-5) ** 2))  # negligible at the faces
    grid = {"E": np.zeros((nz, ny, nx, 4), np.float32), "x0": 0.0, "y0": 0.0, "z0": 0.0, "dx": dx}
    grid["E"][..., 2] = 3e6
    tab = _tab(alpha=2e-20, eta=2e-21)
    ne, npo, nne, info = FL.fluid_run(grid, blob, blob.copy(), np.zeros_like(blob), tab, GAS_N, 5, 1e-11)
    q0 = 0.0
    q1 = float(np.sum(npo) - np.sum(ne) - np.sum(nne))
    assert abs(q1 - q0) <= 1e-9 * float(np.sum(npo))
    assert np.sum(npo) > np.sum(blob) and np.sum(nne) > 0 and len(info["dt"]) == 5
    # electrons drift against the field (towards -z)
    zc = lambda d: float(np.sum(d * z) / np.sum(d))
    assert zc(ne) < zc(blob)
