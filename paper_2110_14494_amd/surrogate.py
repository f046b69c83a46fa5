"""Python handles for the coefficient surrogate entry points (pcmcc_mlp_*).

Argument marshalling only; training, inference, the data set construction and
the held-out fallback decision all run in libpcmcc.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _binding as B


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _vp(a):
    return a.ctypes.data_as(C.c_void_p)


class Norm:
    """Standardisation (and optional fallback description) of the surrogate."""

    def __init__(self, opts: B.pcmcc_mlp_infer_opts | None = None):
        self.opts = opts if opts is not None else B.pcmcc_mlp_infer_opts()
        self._keep = []

    def with_fallback(self, fallback: np.ndarray, cell_lo: float, cell_hi: float, table: np.ndarray,
                      table_lo: float, table_hi: float) -> "Norm":
        fb = np.ascontiguousarray(fallback, dtype=np.uint8)
        tb = _f32(table)
        o = B.pcmcc_mlp_infer_opts()
        C.memmove(C.byref(o), C.byref(self.opts), C.sizeof(o))
        o.n_cells, o.cell_lo, o.cell_hi, o.fallback = fb.size, cell_lo, cell_hi, _vp(fb)
        o.n_nodes, o.table_lo, o.table_hi, o.table = tb.shape[0], table_lo, table_hi, _vp(tb)
        n = Norm(o)
        n._keep = [fb, tb]
        return n


def dataset(EN_Td, values, errors, gas_N: float, max_rel_err: float = 0.1, norm: Norm | None = None,
            ln_floor: float = -200.0):
    """Swarm results -> (x, t, mask, ln, sig, norm) through pcmcc_mlp_dataset
    (sig: the standard error of each ln value, NaN where masked)."""
    EN = np.ascontiguousarray(EN_Td, dtype=np.float64)
    n = EN.size
    res = (B.pcmcc_swarm_result * n)()
    for i in range(n):
        res[i].value[:] = [float(v) for v in values[i]]
        res[i].error[:] = [float(v) for v in errors[i]]
    nm = norm if norm is not None else Norm()
    x = np.zeros(n, np.float32)
    t = np.zeros((n, 6), np.float32)
    m = np.zeros((n, 6), np.float32)
    ln = np.zeros((n, 6), np.float32)
    sig = np.zeros((n, 6), np.float32)
    B.check(B.lib().pcmcc_mlp_dataset(n, _vp(EN), res, float(gas_N), float(max_rel_err),
                                      0 if norm is not None else 1, C.byref(nm.opts), _vp(x), _vp(t), _vp(m),
                                      _vp(ln), _vp(sig), float(ln_floor)))
    return x, t, m, ln, sig, nm


def grad(ctx, params, x, t, mask):
    params, x, t, mask = _f32(params), _f32(x), _f32(t), _f32(mask)
    g = np.zeros(B.MLP_PARAMS, np.float32)
    loss = C.c_double()
    B.check(B.lib().pcmcc_mlp_grad(ctx.h, _vp(params), x.size, _vp(x), _vp(t), _vp(mask), _vp(g), C.byref(loss)),
            ctx.h)
    return loss.value, g


def train(ctx, params0, x, t, mask, epochs: int, lr0: float = 3e-3, lr_min: float = 1e-5, beta1: float = 0.9,
          beta2: float = 0.999, eps: float = 1e-8):
    params0, x, t, mask = _f32(params0), _f32(x), _f32(t), _f32(mask)
    out = np.zeros(B.MLP_PARAMS, np.float32)
    hist = np.zeros(epochs, np.float32)
    st = B.pcmcc_stats()
    o = B.pcmcc_mlp_train_opts(int(epochs), lr0, lr_min, beta1, beta2, eps)
    B.check(B.lib().pcmcc_mlp_train(ctx.h, _vp(params0), x.size, _vp(x), _vp(t), _vp(mask), C.byref(o), _vp(out),
                                    _vp(hist), C.byref(st)), ctx.h)
    return out, hist, st.as_dict()


def infer(ctx, params, norm: Norm, EN: torch.Tensor, out: torch.Tensor | None = None):
    """EN: device float32 [n] (Td) -> device float32 [6, n] ln coefficients."""
    params = _f32(params)
    n = EN.numel()
    if out is None:
        out = torch.empty((6, n), dtype=torch.float32, device=EN.device)
    st = B.pcmcc_stats()
    B.check(B.lib().pcmcc_mlp_infer(ctx.h, _vp(params), C.byref(norm.opts), n, C.c_void_p(EN.data_ptr()),
                                    C.c_void_p(out.data_ptr()), C.byref(st)), ctx.h)
    return out, st.as_dict()


def fallback(ctx, params, norm: Norm, EN_held, ln_held, mask_held, tol_ln: float, n_cells: int, cell_lo: float,
             cell_hi: float, sig_held=None, z_sig: float = 0.0):
    params = _f32(params)
    EN = np.ascontiguousarray(EN_held, dtype=np.float64)
    ln, m = _f32(ln_held), _f32(mask_held)
    sig = None if sig_held is None else _f32(sig_held)
    fb = np.zeros(n_cells, np.uint8)
    err = np.zeros((EN.size, 6), np.float32)
    B.check(B.lib().pcmcc_mlp_fallback(ctx.h, _vp(params), C.byref(norm.opts), EN.size, _vp(EN), _vp(ln), _vp(m),
                                       None if sig is None else _vp(sig), float(tol_ln), float(z_sig), int(n_cells),
                                       float(cell_lo), float(cell_hi), _vp(fb), _vp(err)), ctx.h)
    return fb, err
