"""Removal and splitting of Gaussians (Sec. 8) through the C ABI (host arrays).

The per-Gaussian mean loss over a batch of rays runs on the GPU (Scene.split_statistic /
Batch.split_statistic); these helpers turn it, and the weights, into the removal and split
decisions and form the split Gaussians.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib


def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def prune_mask(weights, z: float = 2.0) -> np.ndarray:
    """True where weight <= mean - z std (Gaussians that contribute minimally)."""
    w = _f32(weights).reshape(-1)
    out = np.empty(w.shape[0], dtype=np.uint8)
    _lib.call("fmb_prune_mask", int(w.shape[0]), _ptr(w), ctypes.c_float(z), _ptr(out))
    return out.astype(bool)


def split_mask(lbar, z: float = 1.0) -> np.ndarray:
    """True where the mean loss lbar >= mean + z std (Gaussians given too much responsibility)."""
    x = _f32(lbar).reshape(-1)
    out = np.empty(x.shape[0], dtype=np.uint8)
    _lib.call("fmb_split_mask", int(x.shape[0]), _ptr(x), ctypes.c_float(z), _ptr(out))
    return out.astype(bool)


def split_gaussians(means, prec, weights, colors=None, noise_w=None, noise_c=None) -> dict:
    """Two Gaussians per given one (rows 2i and 2i + 1); noise_w [2n] and noise_c [2n,3] are the
    caller's draws added in log-weight and unconstrained-colour space (zero if None)."""
    m = _f32(means)
    n = m.shape[0]
    p = _f32(prec, (n, 6))
    w = _f32(weights, (n,))
    c = None if colors is None else _f32(colors, (n, 3))
    nw = _f32(np.zeros(2 * n) if noise_w is None else noise_w, (2 * n,))
    nc = None if c is None else _f32(np.zeros((2 * n, 3)) if noise_c is None else noise_c, (2 * n, 3))
    out = {"means": np.empty((2 * n, 3), np.float32), "prec": np.empty((2 * n, 6), np.float32),
           "weights": np.empty(2 * n, np.float32),
           "colors": None if c is None else np.empty((2 * n, 3), np.float32)}
    _lib.call("fmb_split_gaussians", n, _ptr(m), _ptr(p), _ptr(w), _ptr(c), _ptr(nw), _ptr(nc),
              _ptr(out["means"]), _ptr(out["prec"]), _ptr(out["weights"]), _ptr(out["colors"]))
    return out


def apply_split(means, prec, weights, colors=None, remove: Optional[np.ndarray] = None,
                split: Optional[np.ndarray] = None, rng: Optional[np.random.Generator] = None,
                eps_w: float = 0.1, eps_c: float = 0.1) -> dict:
    """New parameter set: Gaussians marked `remove` dropped, those marked `split` (and not
    removed) replaced by their two children, with N(0, eps^2) noise on log-weights and
    unconstrained colours drawn from `rng`."""
    means, prec, weights = (np.asarray(a, np.float32) for a in (means, prec, weights))
    n = means.shape[0]
    remove = np.zeros(n, bool) if remove is None else np.asarray(remove, bool)
    split = np.zeros(n, bool) if split is None else np.asarray(split, bool)
    keep = ~remove & ~split
    sel = split & ~remove
    rng = rng if rng is not None else np.random.default_rng(0)
    k = int(sel.sum())
    nw = eps_w * rng.standard_normal(2 * k)
    nc = eps_c * rng.standard_normal((2 * k, 3)) if colors is not None else None
    ch = split_gaussians(means[sel], prec[sel], weights[sel], None if colors is None else colors[sel], nw, nc)
    out = {"means": np.concatenate([means[keep], ch["means"]]),
           "prec": np.concatenate([prec[keep], ch["prec"]]),
           "weights": np.concatenate([weights[keep], ch["weights"]])}
    out["colors"] = None if colors is None else np.concatenate([np.asarray(colors, np.float32)[keep], ch["colors"]])
    return out
