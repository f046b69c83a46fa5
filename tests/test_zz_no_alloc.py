"""The allocation-free deposit (pcmcc_deposit_noalloc) against pcmcc_deposit.

Both are called through the C ABI on the same device arrays; the grids must
be equal bit for bit (an integer sum).  Calls follow each other on one GPU
with shrinking inputs (the shared scratch keeps the previous call's contents),
cover the direct and the binned schedule, the largest accepted input, the
rejection beyond it (rho untouched), and a range error followed by a clean
call (the range flag is cleared per call).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2110_14494_amd import workloads as W

pytestmark = pytest.mark.gpu

MAX_N = 2 ** 21


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_14494_amd import pic as P
    return P


def _parts(n, centre, sigma, seed):
    return W.gaussian_particles(n, centre, sigma, seed=seed, weight_seed=seed + 1, log_weight_max=np.log(64.0))


def _both(P, ctx, parts, grid):
    dp = P.Particles.from_numpy(parts)
    dg = P.DeviceGrid(grid)
    ref = dg.zeros_rho()
    got = dg.zeros_rho()
    rc_ref = ctx.deposit(dp, dg, ref, check=False)
    print(f"[gpu] deposit_noalloc n={parts['x'].size} grid={grid['E'].shape[:3]}", flush=True)
    rc = ctx.deposit(dp, dg, got, check=False, no_alloc=True)
    return rc_ref, ref, rc, got


def test_noalloc_deposit_matches_deposit_on_calls_in_a_row(pic):
    ctx = pic.Context(0)
    grid = W.uniform_grid(128, 39e-6, (0.0, 0.0, 0.0))
    c = 64 * 39e-6
    for k, n in enumerate((1_500_000, 300_001, 50_003, 1)):
        parts = _parts(n, (c, c, c), 0.6e-3, seed=40 + k)
        rc_ref, ref, rc, got = _both(pic, ctx, parts, grid)
        assert rc_ref == 0 and rc == 0
        assert torch.equal(ref, got), n
        if n == 50_003:  # and the definition itself, on the CPU
            assert np.array_equal(got.cpu().numpy(), oracle.deposit(parts["x"], parts["y"], parts["z"],
                                                                     parts["w"], grid))
    ctx.close()


def test_noalloc_deposit_limits_and_errors(pic):
    ctx = pic.Context(0)
    # the largest accepted input: 2^21 particles on a 512^3 grid (2^18 tiles)
    grid = W.uniform_grid(512, 20e-6, (0.0, 0.0, 0.0))
    c = 256 * 20e-6
    parts = _parts(MAX_N, (c, c, c), 1.5e-3, seed=50)
    rc_ref, ref, rc, got = _both(pic, ctx, parts, grid)
    assert rc_ref == 0 and rc == 0 and torch.equal(ref, got)
    total = int(got.sum().item())
    assert total == int(np.rint(np.ldexp(parts["w"].astype(np.float64), 32)).astype(np.int64).sum())
    del ref, got
    # one particle more is rejected and leaves rho as it was
    small = W.uniform_grid(64, 39e-6, (0.0, 0.0, 0.0))
    parts = _parts(MAX_N + 1, (32 * 39e-6,) * 3, 0.4e-3, seed=51)
    dp = pic.Particles.from_numpy(parts)
    dg = pic.DeviceGrid(small)
    rho = dg.zeros_rho()
    rho.fill_(7)
    rc = ctx.deposit(dp, dg, rho, check=False, no_alloc=True)
    assert rc == -1 and "maximum" in ctx.last_error()
    assert bool((rho == 7).all())
    # a grid of more than 2^18 tiles (520^3 cells: 65^3 tiles) is rejected too
    dgb = pic.DeviceGrid(W.uniform_grid(8, 1e-5))
    dgb.E = torch.zeros((520, 520, 520, 4), dtype=torch.float32, device="cuda")
    dgb.nx = dgb.ny = dgb.nz = 520
    rho_big = dgb.zeros_rho()
    rho_big.fill_(7)
    parts = _parts(1000, (2.6e-3, 2.6e-3, 2.6e-3), 1e-4, seed=52)
    dp = pic.Particles.from_numpy(parts)
    rc = ctx.deposit(dp, dgb, rho_big, check=False, no_alloc=True)
    assert rc == -1 and "tiles" in ctx.last_error()
    assert bool((rho_big == 7).all())
    del rho_big, dgb
    # a weight outside [0, 2^31) is a range error, and the next call is clean
    parts = _parts(300_000, (32 * 39e-6,) * 3, 0.4e-3, seed=53)
    parts["w"][123] = 2.0 ** 31
    dp = pic.Particles.from_numpy(parts)
    rho = dg.zeros_rho()
    assert ctx.deposit(dp, dg, rho, check=False, no_alloc=True) == -8
    parts["w"][123] = 3.0
    rc_ref, ref, rc, got = _both(pic, ctx, parts, small)
    assert rc_ref == 0 and rc == 0 and torch.equal(ref, got)
    ctx.close()
