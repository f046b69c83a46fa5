"""Host-side code of the library that needs no device: the surrogate's data
set construction (pcmcc_mlp_dataset), checked against its definition in the
header (selected coefficients, ln, masks of unresolved values, the
standardisation and the relative errors)."""
import numpy as np


def test_library_dataset_construction():
    # pcmcc_mlp_dataset is host code in the library (no device work).
    from paper_2110_14494_amd import surrogate as S
    from paper_2110_14494_amd import _binding as B
    n = 40
    EN = np.geomspace(10, 1000, n)
    rng = np.random.default_rng(3)
    vals = np.abs(rng.normal(1.0, 0.2, (n, B.SWARM_NQ))) + 0.1
    errs = 0.01 * vals
    vals[3, 11] = 0.0  # alpha = 0: masked
    errs[5, 12] = 0.5 * vals[5, 12]  # eta unresolved: masked
    vals[7, 2] = np.nan
    N = 2.45e25
    x, t, m, ln, sig, norm = S.dataset(EN, vals, errs, N, max_rel_err=0.1)
    q = {k: i for i, k in enumerate(B.SWARM_QUANTITIES)}
    ref = np.stack([vals[:, q["mu"]] * N, vals[:, q["DL_flux"]] * N, vals[:, q["alpha"]] / N,
                    vals[:, q["eta"]] / N, vals[:, q["mean_eps"]], vals[:, q["bulk_flux_ratio"]]], axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        lr = np.log(ref)
    ok = np.isfinite(lr)
    ok[5, 3] = False
    assert np.array_equal(m.astype(bool), ok)
    o = norm.opts
    assert abs(o.mu_x - np.log(EN).mean()) < 1e-12 and abs(o.sd_x - np.log(EN).std(ddof=1)) < 1e-12
    for k in range(6):
        col = lr[ok[:, k], k]
        assert abs(o.mu_y[k] - col.mean()) < 1e-9 and abs(o.sd_y[k] - col.std(ddof=1)) < 1e-9
        np.testing.assert_allclose(t[ok[:, k], k], (col - o.mu_y[k]) / o.sd_y[k], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(x, (np.log(EN) - o.mu_x) / o.sd_x, rtol=1e-6, atol=1e-6)
    assert np.all(ln[~ok] == -200.0)
    # standard errors of the ln values: relative batch-means errors (1 %)
    assert np.all(np.isnan(sig[~ok]))
    np.testing.assert_allclose(sig[ok], 0.01, rtol=1e-6)
