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


# Rays a scene covers: oracle alpha at least this (per-pixel gates apply there).
HIT_ALPHA = 1e-3
# Floor of the per-pixel relative flow error (pixels) and of the per-entry relative gradient
# error (fraction of the tensor's largest reference entry).
FLOW_FLOOR_PX = 1e-2
GRAD_FLOOR = 1e-3


def per_element_max(a, b, floor):
    """max over elements (rows, for vectors: Euclidean norm per row) of |a - b| / max(|b|, floor)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if b.size == 0:
        return 0.0
    if b.ndim > 1:
        err, mag = np.linalg.norm(a - b, axis=-1), np.linalg.norm(b, axis=-1)
    else:
        err, mag = np.abs(a - b), np.abs(b)
    return float(np.max(err / np.maximum(mag, floor)))


def compare_forward(outs, ref, rays=None, flow=True, normals=True):
    """Errors of GPU outputs (optionally at sampled rays) against oracle outputs: the contract's
    norm-wise (depth, normal, flow) and max absolute (alpha) errors, and per-pixel maxima under
    keys with '@': relative depth over all rays and over rays the scene covers (oracle alpha >=
    HIT_ALPHA), the per-pixel normal error |n - n*| and relative flow error (floor FLOW_FLOOR_PX)."""
    sel = (lambda a: a) if rays is None else (lambda a: a[rays])
    d = sel(to_np(outs["depth"]))
    hit = np.asarray(ref["alpha"]) >= HIT_ALPHA
    e = {"depth": normwise(d, ref["depth"]),
         "alpha": maxabs(sel(to_np(outs["alpha"])), ref["alpha"]),
         "depth@px": per_element_max(d, ref["depth"], 1e-30),
         "depth@px_hit": per_element_max(d[hit], ref["depth"][hit], 1e-30)}
    if normals and outs.get("normal") is not None:
        nr = sel(to_np(outs["normal"]))
        e["normal"] = normwise(nr, ref["normal"])
        e["normal@px"] = per_element_max(nr, ref["normal"], 1.0)
        e["normal@px_hit"] = per_element_max(nr[hit], ref["normal"][hit], 1.0)
    if flow and outs.get("flow") is not None and ref.get("flow") is not None:
        fl = sel(to_np(outs["flow"]))
        e["flow"] = normwise(fl, ref["flow"])
        e["flow@px"] = per_element_max(fl, ref["flow"], FLOW_FLOOR_PX)
        e["flow@px_hit"] = per_element_max(fl[hit], ref["flow"][hit], FLOW_FLOOR_PX)
    return e


def assert_forward(e, what="", per_pixel=True):
    """The contract's norm-wise and max-abs gates; with `per_pixel`, also the relative depth of every
    ray the scene covers within TOL_REL (not for scenes whose blended depth can cancel to near zero,
    e.g. Gaussians on both sides of the camera)."""
    assert e["depth"] <= TOL_REL, f"{what} depth {e}"
    if per_pixel:
        assert e.get("depth@px_hit", 0.0) <= TOL_REL, f"{what} per-pixel depth {e}"
    assert e["alpha"] <= TOL_ALPHA, f"{what} alpha {e}"
    if "normal" in e:
        assert e["normal"] <= TOL_REL, f"{what} normal {e}"
    if "flow" in e:
        assert e["flow"] <= TOL_REL, f"{what} flow {e}"


def compare_grads(g, gref):
    """Norm-wise relative gradient errors per parameter tensor (the contract), and per-entry
    maxima of |g - g*| / max(|g*|, GRAD_FLOOR max|g*|) under keys with '@'."""
    e = {}
    for k in ("means", "prec", "weights", "betas"):
        a, b = to_np(g[k]), np.asarray(gref[k], np.float64)
        e[k] = normwise(a, b)
        scale = float(np.max(np.abs(b))) if b.size else 0.0
        e[k + "@max"] = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), GRAD_FLOOR * scale + 1e-300))) \
            if b.size else 0.0
    return e


def assert_grads(e, what=""):
    for k, v in e.items():
        if "@" not in k:
            assert v <= TOL_GRAD, f"{what} grad {k}: {e}"


def fmt(e):
    """Compact error dictionary for the test log."""
    return "{" + ", ".join(f"{k}: {v:.2e}" for k, v in e.items()) + "}"


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
