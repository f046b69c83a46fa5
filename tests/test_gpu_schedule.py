"""Launch schedule of the step kernel: block size, blocks per compute unit,
refill threshold and work-counter chunk change the time of a step call,
never its results (random numbers follow the electron ids), and the tuner
leaves its input unchanged and stores what it chose."""
import os

import numpy as np
import pytest
import torch

from paper_2110_14494_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_14494_amd import pic as P
    return P


def _by_id(d):
    o = np.argsort(d["id"])
    return {k: v[o] for k, v in d.items()}


def _run(P, cfg, sched, steps=8):
    ctx = P.Context(0)
    ctx.setup(cfg["species"], cfg["tables"])
    if sched is not None:
        ctx.set_schedule(**sched)
    n = cfg["parts"]["x"].size
    dp = P.Particles.from_numpy(cfg["parts"], 32 * n)
    dg = P.DeviceGrid(cfg["grid"])
    rho = dg.zeros_rho()
    print(f"[gpu] schedule {sched} n={n} steps={steps}", flush=True)
    rc, st = ctx.push_collide_deposit(dp, dg, cfg["dt"], steps, cfg["seed"], rho=rho, check=False)
    out = _by_id(dp.to_numpy())
    ctx.close()
    assert rc == 0 and st["majorant_violations"] == 0
    return out, rho.cpu().numpy(), st


COUNTS = ("n", "steps_done", "particle_steps", "trials", "null", "elastic", "excitation", "ionization",
          "attachment", "lost")


def test_schedules_give_identical_results(pic):
    # the tip block: births, attachment, a field that varies cell to cell
    cfg = W.tip_block_config(m=64, n=16384)
    ref, rho_ref, st_ref = _run(pic, cfg, None)
    assert st_ref["ionization"] > 1000
    for s in ({"block": 64, "refill_min": 16, "chunk": 64}, {"block": 256, "blocks_per_cu": 1, "chunk": 4096},
              {"block": 512, "refill_min": 32, "chunk": 128}, {"block": 128, "refill_min": 24}):
        g, rho, st = _run(pic, cfg, s)
        assert st["launch_block"] == s["block"]
        if "refill_min" in s:
            assert st["launch_refill"] == s["refill_min"]
        if "chunk" in s:
            assert st["launch_chunk"] == s["chunk"]
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (s, k)
        assert np.array_equal(rho_ref, rho)
        for k in COUNTS:
            assert st[k] == st_ref[k], (s, k)


def test_default_schedule_and_invalid_values(pic):
    from paper_2110_14494_amd import _binding as B
    cfg = W.plain_swarm_config(n=100)
    ctx = pic.Context(0)
    ctx.setup(cfg["species"], cfg["tables"])
    d = ctx.get_schedule()
    # the most resident waves per compute unit, then the defaults
    assert d["block"] in (64, 128, 256, 512) and d["blocks_per_cu"] >= 1
    assert d["refill_min"] == 24 and d["chunk"] == 512
    for bad in ({"block": 96}, {"refill_min": 20}, {"chunk": 100}, {"chunk": 8192}, {"blocks_per_cu": -1}):
        with pytest.raises(B.PcmccError) as e:
            ctx.set_schedule(**bad)
        assert e.value.code == B.PCMCC_EINVAL
    # more blocks per compute unit than fit: an error at the step call, not a fault
    ctx.set_schedule(block=512, blocks_per_cu=32)
    dp = pic.Particles.from_numpy(cfg["parts"], 1000)
    dg = pic.DeviceGrid(cfg["grid"])
    rc, _ = ctx.push_collide_deposit(dp, dg, cfg["dt"], 1, 0, check=False)
    assert rc == B.PCMCC_EINVAL
    ctx.set_schedule()
    assert ctx.get_schedule() == d
    ctx.close()


def test_largest_tables_fit(pic):
    # eight processes on 1820 energies: the largest tables the step kernel
    # stages in LDS; the schedule resolves to a shape that fits and gives the
    # same electrons as the smallest block
    cfg = W.plain_swarm_config(n=3000)
    t = W.air_like_tables(n_e=1820)
    t["kind"] = np.concatenate([t["kind"], t["kind"]])
    t["threshold"] = np.concatenate([t["threshold"], t["threshold"]])
    t["sigma"] = np.concatenate([t["sigma"], 0.5 * t["sigma"]])
    cfg["tables"] = t
    a, ra, sa = _run(pic, cfg, None, steps=5)
    b, rb, sb = _run(pic, cfg, {"block": 64}, steps=5)
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(ra, rb) and sa["trials"] == sb["trials"]


def test_autotune_leaves_input_and_caches(pic, tmp_path):
    cfg = W.tip_block_config(m=64, n=8192)
    ctx = pic.Context(0)
    ctx.setup(cfg["species"], cfg["tables"])
    n = cfg["parts"]["x"].size
    dp = pic.Particles.from_numpy(cfg["parts"], 32 * n)
    dg = pic.DeviceGrid(cfg["grid"])
    before = dp.to_numpy()
    path = str(tmp_path / "tune.json")
    print("[gpu] autotune_steps", flush=True)
    rc, chosen, t_ms, d_ms = ctx.autotune_steps(dp, dg, cfg["dt"], 3, cfg["seed"], tune_cache=path)
    assert rc == 0 and t_ms > 0 and d_ms > 0 and t_ms <= d_ms
    after = dp.to_numpy()
    for k in before:
        assert np.array_equal(before[k], after[k])
    assert ctx.get_schedule() == chosen
    assert os.path.exists(path) and "k_pic_steps" in open(path).read()
    # a second context takes the stored schedule without timing
    ctx2 = pic.Context(0)
    ctx2.setup(cfg["species"], cfg["tables"])
    rc, chosen2, t2, d2 = ctx2.autotune_steps(dp, dg, cfg["dt"], 3, cfg["seed"], tune_cache=path)
    assert rc == 0 and chosen2 == chosen and t2 == 0 and d2 == 0
    # and the tuned schedule gives the default schedule's electrons
    rc, st = ctx2.push_collide_deposit(dp, dg, cfg["dt"], 4, cfg["seed"])
    tuned = _by_id(dp.to_numpy())
    ctx2.close()
    dp2 = pic.Particles.from_numpy(cfg["parts"], 32 * n)
    ctx.set_schedule()
    ctx.push_collide_deposit(dp2, dg, cfg["dt"], 4, cfg["seed"])
    ref = _by_id(dp2.to_numpy())
    ctx.close()
    for k in ref:
        assert np.array_equal(ref[k], tuned[k])


def test_start_order_does_not_matter(pic):
    # 2^20 electrons over 8 or 9 steps: the call sorts them by tile before
    # the first step; the same electrons in another order give the same
    # electrons by id, the same densities and counters (odd and even step
    # counts: the sort lands in the scratch buffer or is copied back; and a
    # 3-step call, which keeps the given order)
    cfg = W.tip_block_config(m=64, n=2 ** 20)
    perm = np.random.default_rng(3).permutation(cfg["parts"]["x"].size)
    shuffled = dict(cfg, parts={k: v[perm] for k, v in cfg["parts"].items()})
    for steps in (8, 9, 3):
        a, ra, sa = _run(pic, cfg, None, steps=steps)
        b, rb, sb = _run(pic, shuffled, None, steps=steps)
        assert len(np.unique(a["id"])) == a["id"].size
        for k in a:
            assert np.array_equal(a[k], b[k]), (steps, k)
        assert np.array_equal(ra, rb)
        for k in COUNTS:
            assert sa[k] == sb[k], (steps, k)
