"""Flux and bulk swarm coefficients from sampled moments (test infrastructure).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain NumPy FP64.

Definitions (arXiv:2110.14494, Sec. 2.2.2: flux coefficients describe the
mean motion of individual electrons, bulk coefficients the motion of the
centre of mass of the whole group, which differs when ionization or
attachment depends on position through the energy):
  flux drift      W_flux  = -<v_z>                 (time mean over the window)
  bulk drift      W_bulk  = -d<z>/dt               (least-squares slope)
  flux long. diff DL_flux = <(z - <z>)(v_z - <v_z>)>
  bulk long. diff DL_bulk = (1/2) d var(z)/dt
  flux tr. diff   DT_flux = (1/2) <dx dv_x + dy dv_y>
  bulk tr. diff   DT_bulk = (1/4) d (var x + var y)/dt
  rates           nu_ion, nu_att = <nu_k(eps)> (time means of the rate functions)
  growth          nu_eff  = d ln(N 2^L)/dt         (temporal growth, L = weight scale)
  mean energy, mobility mu = W_flux / E, alpha = nu_ion / W_flux,
  eta = nu_att / W_flux, and W_bulk / W_flux.
The field points along +z, so electrons drift along -z and drifts are given
along -E.  Errors: batch means over n_batches contiguous sub-windows.
"""
from __future__ import annotations

import numpy as np

QUANTITIES = ("W_flux", "W_bulk", "DL_flux", "DL_bulk", "DT_flux", "DT_bulk", "nu_ion", "nu_att",
              "nu_eff", "mean_eps", "mu", "alpha", "eta", "bulk_flux_ratio")


def _slope(t, y):
    tm, ym = t.mean(), y.mean()
    return np.sum((t - tm) * (y - ym)) / np.sum((t - tm) ** 2)


def _estimate(t, q, E):
    v = {}
    v["W_flux"] = -q["vz"].mean()
    v["W_bulk"] = -_slope(t, q["z"])
    v["DL_flux"] = q["cL"].mean()
    v["DL_bulk"] = 0.5 * _slope(t, q["varz"])
    v["DT_flux"] = 0.5 * q["cT"].mean()
    v["DT_bulk"] = 0.25 * _slope(t, q["varT"])
    v["nu_ion"] = q["ni"].mean()
    v["nu_att"] = q["na"].mean()
    v["nu_eff"] = _slope(t, q["logN"])
    v["mean_eps"] = q["eps"].mean()
    v["mu"] = v["W_flux"] / E
    v["alpha"] = v["nu_ion"] / v["W_flux"]
    v["eta"] = v["nu_att"] / v["W_flux"]
    v["bulk_flux_ratio"] = v["W_bulk"] / v["W_flux"]
    return np.array([v[k] for k in QUANTITIES])


def per_sample(m, counters):
    """Per-sample means from moment sums m[J, 14] and counters[J, 4]."""
    n = m[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        mx, my, mz = m[:, 1] / n, m[:, 2] / n, m[:, 3] / n
        vx, vy, vz = m[:, 6] / n, m[:, 7] / n, m[:, 8] / n
        return {"n": n, "z": mz, "vz": vz,
                "varz": m[:, 5] / n - mz ** 2,
                "varT": m[:, 4] / n - mx ** 2 - my ** 2,
                "cL": m[:, 10] / n - mz * vz,
                "cT": m[:, 9] / n - mx * vx - my * vy,
                "eps": m[:, 11] / n, "ni": m[:, 12] / n, "na": m[:, 13] / n,
                "logN": np.log(n) + counters[:, 1] * np.log(2.0)}


def estimate(moments, counters, dt_sample: float, window_start: float, n_batches: int, E_field):
    """moments [S, J, 14], counters [S, J, 4] -> values [S, 14], errors [S, 14]."""
    S, J, _ = moments.shape
    t = (np.arange(J) + 1) * dt_sample
    j0 = int(np.argmax(t >= window_start * (1 - 1e-12))) if np.any(t >= window_start * (1 - 1e-12)) else J
    E_field = np.broadcast_to(np.asarray(E_field, dtype=np.float64), (S,))
    vals = np.full((S, len(QUANTITIES)), np.nan)
    errs = np.full((S, len(QUANTITIES)), np.nan)
    for s in range(S):
        q = per_sample(moments[s], counters[s])
        if J - j0 < 2 * n_batches or np.any(~(q["n"][j0:] > 0)):
            continue
        win = {k: v[j0:] for k, v in q.items()}
        tw = t[j0:]
        vals[s] = _estimate(tw, win, E_field[s])
        parts = np.array_split(np.arange(tw.size), n_batches)
        b = np.array([_estimate(tw[ix], {k: v[ix] for k, v in win.items()}, E_field[s]) for ix in parts])
        errs[s] = b.std(axis=0, ddof=1) / np.sqrt(n_batches)
    return vals, errs
