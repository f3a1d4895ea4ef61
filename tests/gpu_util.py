"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the FP64 oracle)."""

from __future__ import annotations

import numpy as np

import workloads as W

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


def custom_scene(n, views, seed, behind=False, flow=False, s_range=(0.05, 0.2)):
    """n Gaussians uniform in [-1,1]^3 (a third behind the front camera if `behind`), views of the
    given (H, W): a front camera at z = -3, the others on a sphere of radius 3, and, with
    `flow`, a second pose shifted by a small translation."""
    g = np.random.Generator(np.random.PCG64(seed))
    means = g.uniform(-1, 1, (n, 3))
    if behind:
        means[: n // 3, 2] = g.uniform(-6, -3.5, n // 3)  # behind the front camera at z = -3
    sc = W.make_scene(g, n, means, log_s_range=s_range)
    e, k, hw = [], [], []
    for i, (h, wd) in enumerate(views):
        if i == 0:
            e.append(np.concatenate([np.eye(3), [[0.0], [0.0], [3.0]]], axis=1))
        else:
            e.append(W.look_at(3.0 * W.fibonacci_sphere(len(views))[i]))
        k.append([float(h), float(h), wd / 2.0, h / 2.0])
        hw.append([h, wd])
    e = np.array(e, np.float32)
    cams = W.Cameras(e, np.array(k, np.float32), np.array(hw, np.int32))
    if flow:
        eb = e.copy()
        eb[:, :, 3] += np.array([0.03, -0.02, 0.01], np.float32)
        cams.w2c_b, cams.intr_b = eb, cams.intr.copy()
    return sc, cams


def hit_mask_cot(cot, alpha_ref, thr=1e-3):
    """Depth/normal/flow/colour cotangents only on rays that see the scene (oracle alpha >= thr); the
    alpha cotangent everywhere.  Over background rays the blend weights are decided by
    log-density differences of order 1e4 that FP32 cannot resolve (see
    test_background_rays_conditioning)."""
    keep = alpha_ref >= thr
    out = {}
    for k, v in cot.items():
        if v is None or k == "alpha":
            out[k] = v
        else:
            out[k] = (v * keep.reshape(-1, *([1] * (v.ndim - 1)))).astype(np.float32)
    return out
