"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the FP64 oracle)."""

from __future__ import annotations

import numpy as np

# Tolerances of the renderer's contract: norm-wise relative for depth, normals, flow
# and gradients (per tensor), max absolute for alpha.
TOL_REL = 1e-4
TOL_ALPHA = 1e-5
TOL_GRAD = 1e-3


def to_np(t):
    return None if t is None else t.detach().cpu().double().numpy()


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)))) if np.size(b) else 0.0


def make_scene(fmb, torch, sc, cams, betas, eta, dev):
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev).contiguous()  # noqa: E731
    params = (t(sc.means), t(sc.prec), t(sc.weights), t(np.asarray(betas, np.float32)))
    c = fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, cams.w2c_b, cams.intr_b, device=dev,
                               w2c_c=cams.w2c_c, intr_c=cams.intr_c)
    return fmb.Scene(*params, eta, c), params


def compare_forward(outs, ref, rays=None, flow=True, normals=True):
    """Errors of GPU outputs (optionally at sampled rays) against oracle outputs."""
    sel = (lambda a: a) if rays is None else (lambda a: a[rays])
    e = {"depth": normwise(sel(to_np(outs["depth"])), ref["depth"]),
         "alpha": maxabs(sel(to_np(outs["alpha"])), ref["alpha"])}
    if normals and outs.get("normal") is not None:
        e["normal"] = normwise(sel(to_np(outs["normal"])), ref["normal"])
    if flow and outs.get("flow") is not None and ref.get("flow") is not None:
        e["flow"] = normwise(sel(to_np(outs["flow"])), ref["flow"])
    return e


def assert_forward(e, what=""):
    assert e["depth"] <= TOL_REL, f"{what} depth {e}"
    assert e["alpha"] <= TOL_ALPHA, f"{what} alpha {e}"
    if "normal" in e:
        assert e["normal"] <= TOL_REL, f"{what} normal {e}"
    if "flow" in e:
        assert e["flow"] <= TOL_REL, f"{what} flow {e}"


def compare_grads(g, gref):
    return {k: normwise(to_np(g[k]), gref[k]) for k in ("means", "prec", "weights", "betas")}


def assert_grads(e, what=""):
    for k, v in e.items():
        assert v <= TOL_GRAD, f"{what} grad {k}: {e}"
