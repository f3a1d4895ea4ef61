"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Full-size workloads render every ray on the GPU in the launch configuration the
benchmark uses; where the oracle cannot render all rays in seconds it is evaluated
on a seeded sample of rays (forward), and the backward pass is driven by cotangents
that are zero except on that sample, so the oracle's gradient over the sample is the
exact reference for the GPU gradient over the whole image.
"""

from __future__ import annotations

import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import (TOL_ALPHA, TOL_GRAD, TOL_REL, assert_forward, assert_grads, compare_forward,
                            compare_grads, custom_scene, fmt, hit_mask_cot, make_scene, maxabs, normwise, to_np)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def fmb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_14737_amd as m
    return m


def _say(*a):
    print(*a, flush=True)


def _sample(n_rays, k, seed):
    if k is None or k >= n_rays:
        return None
    g = np.random.Generator(np.random.PCG64(seed))
    return np.sort(g.choice(n_rays, size=k, replace=False))


FULL = [("fwd64", None), ("fwdbwd128", None), ("flow480", 20000), ("large1080", 3000)]


@pytest.mark.parametrize("name,sample", FULL, ids=[f[0] for f in FULL])
def test_forward_parity(fmb, name, sample):
    w = W.make_config(name)
    sc, cams = w.scenes[0], w.cameras[0]
    _say(f"[fwd] {name}: N={sc.n} P={cams.n_rays} sample={sample}")
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    outs = scene.render(normals=w.normals)
    torch.cuda.synchronize()
    rays = _sample(cams.n_rays, sample, 7)
    ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays)
    e = compare_forward(outs, ref, rays, normals=w.normals)
    _say(f"[fwd] {name}: {e}")
    assert_forward(e, name)
    assert np.all(np.isfinite(to_np(outs["depth"]))) and np.all(np.isfinite(to_np(outs["alpha"])))


BWD = [("fwd64", None), ("fwdbwd128", None), ("flow480", 20000), ("large1080", 2000)]


@pytest.mark.parametrize("name,sample", BWD, ids=[b[0] for b in BWD])
def test_backward_parity(fmb, name, sample):
    w = W.make_config(name)
    sc, cams = w.scenes[0], w.cameras[0]
    p = cams.n_rays
    _say(f"[bwd] {name}: N={sc.n} P={p} sample={sample}")
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    outs = scene.render(normals=w.normals)
    cot = W.random_cotangents(p, 1234, flow=cams.has_flow, normals=w.normals)
    rays = _sample(p, sample, 11)
    if rays is not None:
        mask = np.zeros(p, dtype=bool)
        mask[rays] = True
        for k, v in cot.items():
            if v is not None:
                v[~mask] = 0.0
    t = lambda a: None if a is None else torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]), t(cot["flow"]))
    torch.cuda.synchronize()
    cot_s = {k: (None if v is None else (v if rays is None else v[rays])) for k, v in cot.items()}
    _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays, cot=cot_s)
    e = compare_grads(g, gref)
    _say(f"[bwd] {name}: {e}")
    assert_grads(e, name)


# ---------------------------------------------------------------------------------------
# Ragged and degenerate cases
# ---------------------------------------------------------------------------------------

RAGGED = [
    ("n1_1x1", 1, [(1, 1)]),
    ("n1_odd", 1, [(17, 23)]),
    ("n7_multi", 7, [(5, 3), (64, 64), (1, 1), (33, 65)]),
    ("n129_two_tiles", 129, [(20, 31)]),
    ("n257_chunks", 257, [(40, 50), (3, 7)]),
    ("n600_tiny_img", 600, [(7, 9)]),
]


@pytest.mark.parametrize("label,n,views", RAGGED, ids=[r[0] for r in RAGGED])
def test_ragged_parity(fmb, label, n, views):
    sc, cams = custom_scene(n, views, seed=n, flow=True)
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say(f"[ragged] {label}: N={n} views={views}")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, betas, 1.0)
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 5, flow=True), ref["alpha"])
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]), t(cot["flow"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, betas, 1.0, cot=cot)
    e = compare_forward(outs, ref)
    eg = compare_grads(g, gref)
    _say(f"[ragged] {label}: {e} {eg}")
    assert_forward(e, label)
    assert_grads(eg, label)


@pytest.mark.parametrize("model", ["blend", "composite"])
def test_anisotropic_tile_bounds(fmb, model):
    """Gaussians with scale ratios up to 100 (needles and discs), where the tile bound that lets a
    wave pass over whole (ray tile, Gaussian) pairs is tightest against the true densities: the
    forward and the gradients (depth and alpha cotangents as in the benchmarked step, and random
    cotangents on covered rays) match the oracle in both models."""
    sc, cams = custom_scene(60, [(64, 64), (96, 128), (48, 40)], seed=29, s_range=(0.005, 0.5))
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say(f"[aniso] {model}: N=60 scale ratios up to 100")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    scene.set_model(model)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, betas, 1.0, model=model)
    e = compare_forward(outs, ref, flow=False)
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 31, flow=False), ref["alpha"])
    for c in (dict(cot, normal=None), cot):
        g = scene.backward(outs, t(c["depth"]), t(c["alpha"]), None if c["normal"] is None else t(c["normal"]))
        torch.cuda.synchronize()
        _, gref, _ = O.render_workload_view(sc, cams, betas, 1.0, cot=c, model=model)
        eg = compare_grads(g, gref)
        _say(f"[aniso] {model} normal cotangent {c['normal'] is not None}: {e} {fmt(eg)}")
        assert_grads(eg, f"anisotropic {model}")
    assert_forward(e, f"anisotropic {model}")


def test_background_rays_conditioning(fmb):
    """Unmasked random cotangents on a sparse scene whose image is mostly background.  There the
    exact gradient itself moves by ~1e-3 when the FP32 inputs move by one ulp (measured below
    with the oracle): background pairs have log-densities d of order -1e3..-1e4, and the blend
    weights of Eq. (7) depend on differences of such values.  The kernels hold d in FP32, whose
    rounding (|d| 2^-24) is larger than a one-ulp change of the inputs by about |d| / |x|, so the
    bound is ten times the measured one-ulp sensitivity (and never below the 1e-3 contract)."""
    sc, cams = custom_scene(7, [(5, 3), (64, 64), (1, 1), (33, 65)], seed=7, flow=True)
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say("[background] N=7 sparse scene, unmasked cotangents")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    outs = scene.render(normals=True)
    cot = W.random_cotangents(cams.n_rays, 5, flow=True)
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]), t(cot["flow"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, betas, 1.0, cot=cot)
    rng = np.random.Generator(np.random.PCG64(1))
    sens = {k: 0.0 for k in gref}
    for _ in range(3):
        jit = W.Scene(sc.means.astype(np.float64) * (1 + 2.0 ** -24 * rng.standard_normal(sc.means.shape)),
                      sc.prec.astype(np.float64) * (1 + 2.0 ** -24 * rng.standard_normal(sc.prec.shape)),
                      sc.weights)
        _, gj, _ = O.render_workload_view(jit, cams, betas, 1.0, cot=cot)
        for k in gref:
            sens[k] = max(sens[k], normwise(gj[k], gref[k]))
    eg = compare_grads(g, gref)
    _say(f"[background] gpu {eg} oracle one-ulp sensitivity {sens}")
    for k in ("means", "prec", "weights", "betas"):
        assert eg[k] <= max(TOL_GRAD, 10.0 * sens[k]), (k, eg, sens)


def test_loss_gradient_parity(fmb):
    """Gradient of the workload loss (alpha-weighted L1 depth + BCE alpha against targets rendered
    from the perturbed scene); targets and cotangents come from the oracle's own renders."""
    w = W.make_config("fwdbwd128")
    sc, cams = w.scenes[0], w.cameras[0]
    _say("[loss] fwdbwd128 L1 depth + BCE alpha")
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta)
    tgt, _, _ = O.render_workload_view(w.targets[0], cams, w.betas, w.eta)
    p = cams.n_rays
    gd = tgt["alpha"] * np.sign(ref["depth"] - tgt["depth"]) / p
    a = np.clip(ref["alpha"], 1e-6, 1 - 1e-6)
    inside = (ref["alpha"] >= 1e-6) & (ref["alpha"] <= 1 - 1e-6)
    ga = np.where(inside, (a - tgt["alpha"]) / (a * (1 - a)), 0.0) / p
    cot = {"depth": gd.astype(np.float32), "alpha": ga.astype(np.float32), "normal": None, "flow": None}
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, cot=cot)
    eg = compare_grads(g, gref)
    _say(f"[loss] {eg}")
    assert_grads(eg, "loss")


def test_behind_camera_and_eta(fmb):
    """Gaussians behind the camera (t < 0) are blended like any other (Eq. 7 without clamp);
    a non-unit eta rescales the depth term."""
    sc, cams = custom_scene(30, [(48, 40)], seed=3, behind=True)
    betas = np.array([W.BETA1 * 0.5, W.BETA2], np.float32)
    _say("[behind] N=30, 48x40, eta=2.5")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 2.5, DEV)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, betas, 2.5)
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 9, flow=False), ref["alpha"])
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, betas, 2.5, cot=cot)
    # per pixel, the blend of depths of both signs (Gaussians behind the camera) can cancel to near
    # zero, where the relative depth is ill-conditioned: the norm-wise contract only
    assert_forward(compare_forward(outs, ref), "behind", per_pixel=False)
    assert_grads(compare_grads(g, gref), "behind")


def test_flow_equal_poses_is_zero(fmb):
    sc, cams = custom_scene(20, [(32, 48), (16, 16)], seed=4)
    cams.w2c_b, cams.intr_b = cams.w2c.copy(), cams.intr.copy()
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say("[flow0] equal poses")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    outs = scene.render(normals=False)
    torch.cuda.synchronize()
    assert torch.count_nonzero(outs["flow"]).item() == 0


def test_alpha_interop_value(fmb):
    """A lone Gaussian with lambda = log 80 seen through its mean renders alpha = 79/80."""
    means = np.zeros((1, 3), np.float32)
    prec = np.array([[10.0, 1.0, -2.0, 8.0, 0.5, 12.0]], np.float32)
    sc = W.Scene(means, prec, np.array([math.log(80.0)], np.float32))
    cams = W.Cameras(np.concatenate([np.eye(3), [[0.0], [0.0], [3.0]]], axis=1)[None].astype(np.float32),
                     np.array([[8.0, 8.0, 1.0, 1.0]], np.float32), np.array([[2, 2]], np.int32))
    # pixel (0,0) has its centre at (0.5, 0.5) != principal point (1,1); use principal point (0.5,0.5)
    cams.intr[0, 2:] = 0.5
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say("[interop] alpha 79/80")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    outs = scene.render(normals=True)
    torch.cuda.synchronize()
    assert abs(float(outs["alpha"][0]) - 79.0 / 80.0) <= TOL_ALPHA
    assert abs(float(outs["depth"][0]) - 3.0) <= 3.0 * TOL_REL


def test_validate_flags(fmb):
    sc, cams = custom_scene(8, [(8, 8)], seed=6)
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say("[validate]")
    scene, (m, p, wt, b) = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    assert scene.validate() == 0
    m[2, 1] = float("nan")
    wt[3] = -1.0
    p[4, 3] = 0.0
    assert scene.validate() == 1 | 2 | 4


def test_autograd_matches_backward(fmb):
    w = W.make_config("fwd64")
    sc, cams = w.scenes[0], w.cameras[0]
    _say("[autograd] fwd64")
    scene, (m, p, wt, b) = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    params = [x.clone().requires_grad_(True) for x in (m, p, wt, b)]
    depth, alpha, normal, _, _ = fmb.render(scene, *params, normals=True)
    cot = W.random_cotangents(cams.n_rays, 77, flow=False)
    t = lambda a: torch.as_tensor(a, device=DEV)  # noqa: E731
    loss = (depth * t(cot["depth"])).sum() + (alpha * t(cot["alpha"])).sum() + (normal * t(cot["normal"])).sum()
    loss.backward()
    outs = scene.render(normals=True)
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]))
    torch.cuda.synchronize()
    for x, k in zip(params, ("means", "prec", "weights", "betas")):
        assert torch.equal(x.grad, g[k]), k


def test_autograd_unused_outputs(fmb):
    """Outputs the loss does not use pass no cotangent: a loss of alpha alone equals the
    backward with only an alpha cotangent, bit for bit."""
    w = W.make_config("fwd64")
    sc, cams = w.scenes[0], w.cameras[0]
    _say("[autograd-unused] fwd64")
    scene, (m, p, wt, b) = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    params = [x.clone().requires_grad_(True) for x in (m, p, wt, b)]
    depth, alpha, normal, _, _ = fmb.render(scene, *params, normals=True)
    ga = torch.as_tensor(W.random_cotangents(cams.n_rays, 79, flow=False)["alpha"], device=DEV)
    (alpha * ga).sum().backward()
    outs = scene.render(normals=True)
    g = scene.backward(outs, None, ga.contiguous(), None)
    torch.cuda.synchronize()
    for x, k in zip(params, ("means", "prec", "weights", "betas")):
        assert torch.equal(x.grad, g[k]), k


@pytest.mark.parametrize("with_normals", [True, False], ids=["normals", "depth_alpha"])
def test_finite_differences_on_gpu(fmb, with_normals):
    """Loose sanity check of the adjoint with the GPU alone: central differences of the FP32
    forward pass (loss accumulated in FP64 on the host) against the backward pass, on the
    entries of each parameter tensor with the largest gradients.  With and without a normal
    cotangent (the two forms of the pair adjoint)."""
    w = W.make_config("fwd64")
    sc, cams = w.scenes[0], w.cameras[0]
    _say(f"[fd] fwd64 normals={with_normals}")
    scene, (m, p, wt, b) = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    cot = W.random_cotangents(cams.n_rays, 91, flow=False)
    cd, ca, cn = (torch.as_tensor(cot[k], device=DEV, dtype=torch.float64) for k in ("depth", "alpha", "normal"))

    def loss():
        o = scene.render(normals=True)
        torch.cuda.synchronize()
        v = (o["depth"].double() * cd).sum() + (o["alpha"].double() * ca).sum()
        if with_normals:
            v = v + (o["normal"].double() * cn).sum()
        return float(v)

    outs = scene.render(normals=True)
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]) if with_normals else None)
    torch.cuda.synchronize()
    worst = 0.0
    for name, x in (("means", m), ("prec", p), ("weights", wt), ("betas", b)):
        gx = g[name].reshape(-1).double().cpu()
        flat = x.view(-1)
        top = torch.argsort(gx.abs(), descending=True)[:4 if name != "betas" else 2]
        for idx in top.tolist():
            x0 = float(flat[idx])
            # small steps where the loss bends over a Gaussian's width; the blend parameters
            # are smooth and their gradients small, so a larger step keeps FP32 noise down
            h = (1e-3 if name == "betas" else 1e-4) * max(1.0, abs(x0))
            flat[idx] = x0 + h
            xp = float(flat[idx])  # the float32 values actually rendered
            lp = loss()
            flat[idx] = x0 - h
            xm = float(flat[idx])
            lm = loss()
            flat[idx] = x0
            fd = (lp - lm) / (xp - xm)
            rel = abs(fd - float(gx[idx])) / max(abs(float(gx[idx])), 1e-2 * float(gx.abs().max()))
            worst = max(worst, rel)
            _say(f"[fd] {name}[{idx}] fd {fd:.6e} adjoint {float(gx[idx]):.6e} rel {rel:.2e}")
    assert worst <= 2e-2, worst


def test_deterministic_backward(fmb):
    w = W.make_config("fwdbwd128")
    sc, cams = w.scenes[0], w.cameras[0]
    _say("[determinism] fwdbwd128 twice")
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    outs = scene.render(normals=True)
    cot = W.random_cotangents(cams.n_rays, 3, flow=False)
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    g1 = {k: v.clone() for k, v in scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"])).items()
          if v is not None}
    g2 = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]))
    torch.cuda.synchronize()
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k


def test_scene_step_single_graph(fmb):
    """A single scene's step (forward with normals, backward of depth and alpha cotangents,
    finalize) captured from its stream as one graph replays like the eager calls, with eager work
    between the replays."""
    w = W.make_config("fwdbwd128")
    sc, cams = w.scenes[0], w.cameras[0]
    _say("[scene-graph] fwdbwd128")
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    outs = scene.render(normals=True)
    cot = W.random_cotangents(cams.n_rays, 7, flow=False)
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    gd, ga = t(cot["depth"]), t(cot["alpha"])
    grads = scene.backward(outs, gd, ga)

    def step():
        scene.render(normals=True, out=outs)
        scene.backward(outs, gd, ga, grads=grads)

    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        step()
    torch.cuda.current_stream().wait_stream(s2)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in grads.items() if v is not None}
    ref_depth = outs["depth"].clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        outs["depth"].fill_(float("nan"))
        for v in grads.values():
            if v is not None:
                v.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(outs["depth"], ref_depth), rep
        for k, v in ref.items():
            assert torch.equal(grads[k], v), (rep, k)
        step()
        torch.cuda.synchronize()
        _say(f"[scene-graph] replay {rep} matches eager")


@pytest.mark.parametrize("norm", [1, 2])
def test_loss_grad_kernel(fmb, norm):
    """The fused loss-gradient kernel against the oracle's definition of the Sec. 4 loss."""
    g = np.random.Generator(np.random.PCG64(40 + norm))
    p = 10007
    depth = g.uniform(1, 5, p).astype(np.float32)
    depth_t = depth.copy()
    depth_t[::3] = g.uniform(1, 5, len(depth_t[::3])).astype(np.float32)   # some exact ties
    alpha = g.uniform(0, 1, p).astype(np.float32)
    alpha[:5] = [0.0, 1.0, 5e-7, 1 - 1e-7, 1e-6]                              # clamp edges
    alpha_t = (g.uniform(0, 1, p) > 0.4).astype(np.float32)
    flow = g.standard_normal((p, 2)).astype(np.float32)
    flow_t = g.standard_normal((p, 2)).astype(np.float32)
    color = g.uniform(0, 1, (p, 3)).astype(np.float32)
    color_t = g.uniform(0, 1, (p, 3)).astype(np.float32)
    _say(f"[loss-kernel] p={p} norm={norm}")
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    bl = torch.empty((p + 1023) // 1024, device=DEV)
    cot = fmb.loss_grad({"depth": t(depth), "alpha": t(alpha), "flow": t(flow), "color": t(color)}, t(depth_t),
                        t(alpha_t), t(flow_t), w_depth=1.5, w_flow=2.5, flow_norm=norm, block_loss=bl,
                        color_t=t(color_t), w_color=4.5)
    torch.cuda.synchronize()
    L, gref = O.loss_grad(depth, alpha, depth_t, alpha_t, flow, flow_t, 1.5, 2.5, norm, color, color_t, 4.5)
    for k in ("depth", "alpha", "flow", "color"):
        got = to_np(cot[k])
        err = np.abs(got - gref[k])
        assert np.all(err <= 1e-5 * np.abs(gref[k]) + 1e-12), (k, float(err.max()))
    assert abs(float(bl.double().sum()) - L) <= 1e-5 * abs(L)


@pytest.mark.parametrize("model,normals", [("blend", True), ("blend", False), ("composite", True),
                                           ("composite", False)])
def test_explicit_ray_minibatch(fmb, model, normals):
    """A random minibatch of rays across all views (uneven counts, one empty view, sub-pixel
    directions) through fmb_set_rays, against the oracle on the same float32 directions; both
    models, with a normal cotangent and without one (the blend model's tiled backward then takes
    tiles of 64 consecutive rays of the minibatch)."""
    w = W.make_config("flow480")
    sc, cams = w.scenes[0], w.cameras[0]
    g = np.random.Generator(np.random.PCG64(77))
    counts = g.integers(1000, 9000, size=cams.v).astype(np.int32)
    counts[3] = 0
    views = np.repeat(np.arange(cams.v), counts).astype(np.int32)
    p = int(counts.sum())
    # directions through random sub-pixel positions, built in float64 from the camera, then float32
    px = np.stack([g.uniform(0, 640, p), g.uniform(0, 480, p)], axis=1)
    k = cams.intr[views].astype(np.float64)
    dc = np.stack([(px[:, 0] - k[:, 2]) / k[:, 0], (px[:, 1] - k[:, 3]) / k[:, 1], np.ones(p)], axis=1)
    rot = cams.w2c[views, :, :3].astype(np.float64)
    dirs = (np.einsum("pji,pj->pi", rot, dc) * g.uniform(0.5, 2.0, (p, 1))).astype(np.float32)
    _say(f"[minibatch] flow480 {model} normals={normals} views counts={counts.tolist()} P={p}")
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    params = (t(sc.means), t(sc.prec), t(sc.weights), t(w.betas))
    c = fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, cams.w2c_b, cams.intr_b, device=DEV)
    scene = fmb.Scene(*params, w.eta)
    td = t(dirs)
    scene.set_rays(c, counts, td)
    if model == "composite":
        scene.set_model("composite")
    assert scene.n_rays == p
    outs = scene.render(normals=True)
    o, v = O.dir_rays(views, dirs, cams.w2c)
    osc = O.OracleScene.of(sc.means, sc.prec, sc.weights, w.betas, w.eta)
    kw = dict(view=views, w2c_a=cams.w2c, intr_a=cams.intr, w2c_b=cams.w2c_b, intr_b=cams.intr_b, model=model)
    ref = O.render(osc, o, v, **kw)
    cot = hit_mask_cot(W.random_cotangents(p, 12, flow=True, normals=normals), ref["alpha"])
    gn = t(cot["normal"]) if normals else None
    gr = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), gn, t(cot["flow"]))
    torch.cuda.synchronize()
    gref = O.backward(osc, o, v, cot, **kw)
    e = compare_forward(outs, ref)
    eg = compare_grads(gr, gref)
    _say(f"[minibatch] {e} {eg}")
    assert_forward(e, "minibatch")
    assert_grads(eg, "minibatch")


def test_colour_parity(fmb):
    """Per-Gaussian colours (sigmoid of unconstrained parameters, blended by Eq. 3): forward colour
    and the gradients of depth/alpha/normal/colour cotangents, against the oracle."""
    w = W.make_config("fwdbwd128")
    sc, cams = w.scenes[0], w.cameras[0]
    g = np.random.Generator(np.random.PCG64(91))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    _say(f"[colour] fwdbwd128 N={sc.n} P={cams.n_rays}")
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    t = lambda a: torch.as_tensor(a, device=DEV).contiguous()  # noqa: E731
    tq = t(q)
    scene.set_colors(tq)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta, colors=q)
    e = compare_forward(outs, ref)
    e["color"] = normwise(to_np(outs["color"]), ref["color"])
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 31, flow=False), ref["alpha"])
    cot["color"] = (g.standard_normal((cams.n_rays, 3)) * (ref["alpha"] >= 1e-3)[:, None]).astype(np.float32)
    gr = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]), None, g_color=t(cot["color"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, cot=cot, colors=q)
    eg = compare_grads(gr, gref)
    eg["colors"] = normwise(to_np(gr["colors"]), gref["colors"])
    _say(f"[colour] {e} {eg}")
    assert_forward(e, "colour")
    assert e["color"] <= TOL_REL
    assert_grads(eg, "colour")


def test_colour_autograd_and_batch(fmb):
    """Colours through the autograd function, and the batched persistent path with colours equals
    the per-scene path bit for bit."""
    w = W.make_config("batch16")
    idx = [1, 8, 14]
    scenes = [w.scenes[i] for i in idx]
    camsl = [w.cameras[i] for i in idx]
    g = np.random.Generator(np.random.PCG64(92))
    qs = [(1.5 * g.standard_normal((s.n, 3))).astype(np.float32) for s in scenes]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    means = t(np.concatenate([s.means for s in scenes]))
    prec = t(np.concatenate([s.prec for s in scenes]))
    weights = t(np.concatenate([s.weights for s in scenes]))
    betas = t(np.tile(w.betas, (len(scenes), 1)))
    colors = t(np.concatenate(qs))
    cams = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, device=DEV) for c in camsl]
    b = fmb.Batch(means, prec, weights, betas, [w.eta] * len(scenes), [s.n for s in scenes], cams)
    b.set_colors(colors)
    _say(f"[colour-batch] scenes {idx} P={b.n_rays}")
    outs = b.forward(b.alloc_outputs(normals=True, color=True))
    gc = W.random_cotangents(b.n_rays, 93, flow=False)
    cot = {"depth": t(gc["depth"]), "alpha": t(gc["alpha"]), "normal": None, "flow": None,
           "color": t(g.standard_normal((b.n_rays, 3)).astype(np.float32))}
    grads = b.backward(outs, cot, b.alloc_grads(colors=True))
    torch.cuda.synchronize()
    for i in range(len(scenes)):
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        scene = fmb.Scene(means[g0:g1], prec[g0:g1], weights[g0:g1], betas[i], w.eta, cams[i])
        params = [x.clone().requires_grad_(True) for x in (means[g0:g1], prec[g0:g1], weights[g0:g1],
                                                               betas[i], colors[g0:g1])]
        depth, alpha, normal, _, color = fmb.render(scene, *params[:4], normals=True, colors=params[4])
        assert torch.equal(color, outs["color"][r0:r1]) and torch.equal(depth, outs["depth"][r0:r1])
        # the normals are rendered but unused by the loss: no normal cotangent reaches the
        # backward, as in the batched call
        loss = (depth * cot["depth"][r0:r1]).sum() + (alpha * cot["alpha"][r0:r1]).sum() \
            + (color * cot["color"][r0:r1]).sum()
        loss.backward()
        torch.cuda.synchronize()
        for x, k in zip(params, ("means", "prec", "weights", "betas", "colors")):
            ref = grads[k][i] if k == "betas" else grads[k][g0:g1]
            assert torch.equal(x.grad, ref), (i, k)


def test_two_way_flow_and_quality(fmb):
    """Forward and backward flow per ray (Sec. 5) and the direct-intersection quality max_i w_i
    (Sec. 6, read from the stash) against the oracle; the 4-column loss kernel; and the batched
    path with a third pose equal to the per-scene path bit for bit."""
    sc, cams = custom_scene(40, [(48, 64), (33, 17), (1, 5)], seed=44, flow=True)
    cams = W.with_backward_flow(cams, seed=45)
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say(f"[two-way] N=40 P={cams.n_rays}")
    scene, params = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    outs = scene.render(normals=True)
    assert tuple(outs["flow"].shape) == (cams.n_rays, 4)
    ref, _, (view, row, col) = O.render_workload_view(sc, cams, betas, 1.0)
    e = compare_forward(outs, ref)
    e["flow_back"] = normwise(to_np(outs["flow"])[:, 2:], ref["flow"][:, 2:])
    # quality on a sample of rays, one oracle ray at a time
    rs = _sample(cams.n_rays, 400, 46)
    o, v = O.pixel_rays(view[rs], row[rs], col[rs], cams.w2c, cams.intr)
    osc = O.OracleScene.of(sc.means, sc.prec, sc.weights, betas, 1.0)
    q_ref = O.max_weight(osc, o, v)
    q = to_np(fmb.Scene.quality(outs))[rs]
    # compared where the ray sees the scene: over background rays the weights are decided by
    # log-density differences FP32 cannot resolve (as for the gradients there)
    hit = ref["alpha"][rs] >= 1e-3
    assert hit.sum() >= 100
    e["quality"] = float(np.max(np.abs(q - q_ref)[hit]))
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 47, flow=True), ref["alpha"])
    g = np.random.Generator(np.random.PCG64(48))
    cot["flow"] = (g.standard_normal((cams.n_rays, 4)) * (ref["alpha"] >= 1e-3)[:, None]).astype(np.float32)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    gr = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]), t(cot["flow"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, betas, 1.0, cot=cot)
    eg = compare_grads(gr, gref)
    _say(f"[two-way] {e} {eg}")
    assert_forward(e, "two-way")
    assert e["flow_back"] <= TOL_REL
    assert e["quality"] <= TOL_REL
    assert_grads(eg, "two-way")
    # loss over both flows
    flow_t = g.standard_normal((cams.n_rays, 4)).astype(np.float32)
    alpha_t = (ref["alpha"] > 0.5).astype(np.float32)
    depth_t = (to_np(outs["depth"]) + g.uniform(-0.1, 0.1, cams.n_rays)).astype(np.float32)
    lc = fmb.loss_grad(outs, t(depth_t), t(alpha_t), t(flow_t), w_flow=0.5, flow_norm=2)
    torch.cuda.synchronize()
    _, lref = O.loss_grad(to_np(outs["depth"]), to_np(outs["alpha"]), depth_t, alpha_t,
                          to_np(outs["flow"]), flow_t, 1.0, 0.5, 2)
    err = np.abs(to_np(lc["flow"]) - lref["flow"])
    assert np.all(err <= 1e-5 * np.abs(lref["flow"]) + 1e-12), float(err.max())
    # batched persistent path with the third pose: identical to the per-scene path
    c = fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, cams.w2c_b, cams.intr_b, device=DEV,
                               w2c_c=cams.w2c_c, intr_c=cams.intr_c)
    b = fmb.Batch(*params, [1.0], [sc.n], [c])
    bo = b.forward(b.alloc_outputs(normals=True))
    torch.cuda.synchronize()
    for k in ("depth", "alpha", "normal", "flow", "stash"):
        assert torch.equal(bo[k], outs[k]), k


VARIANT_CASES = [
    ("n7_multi", 7, [(5, 3), (64, 64), (1, 1), (33, 65)]),
    ("n90", 90, [(37, 41)]),
    ("n257", 257, [(40, 50), (3, 7)]),
    ("n600", 600, [(12, 20)]),  # a ray-lane item's chunk (the whole scene) above 256 Gaussians
]


@pytest.mark.parametrize("variant", range(9))
@pytest.mark.parametrize("label,n,views", VARIANT_CASES, ids=[c[0] for c in VARIANT_CASES])
def test_backward_variants(fmb, variant, label, n, views):
    """Every backward variant (Gaussian-lane 0-2, ray-lane 3-5, tiled 6-8, which hand a normal
    cotangent to variant 2) against the oracle, with normal, flow (both directions) and colour
    cotangents."""
    sc, cams = custom_scene(n, views, seed=300 + n, flow=True)
    cams = W.with_backward_flow(cams, seed=301)
    g = np.random.Generator(np.random.PCG64(302))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    _say(f"[variant] {label} bwd variant {variant}: N={n} views={views}")
    scene, _ = make_scene(fmb, torch, sc, cams, np.array([W.BETA1, W.BETA2], np.float32), 1.0, DEV)
    fmb.set_launch_config(scene=scene, bwd_variant=variant)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    scene.set_colors(t(q))
    outs = scene.render(normals=True)
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    ref, _, _ = O.render_workload_view(sc, cams, betas, 1.0, colors=q)
    hit = ref["alpha"] >= 1e-3
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 303, flow=False), ref["alpha"])
    cot["flow"] = (g.standard_normal((cams.n_rays, 4)) * hit[:, None]).astype(np.float32)
    cot["color"] = (g.standard_normal((cams.n_rays, 3)) * hit[:, None]).astype(np.float32)
    gr = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), t(cot["normal"]), t(cot["flow"]),
                        g_color=t(cot["color"]))
    torch.cuda.synchronize()
    assert fmb.launch_config(scene=scene)["bwd_variant"] == variant
    _, gref, _ = O.render_workload_view(sc, cams, betas, 1.0, cot=cot, colors=q)
    eg = compare_grads(gr, gref)
    eg["colors"] = normwise(to_np(gr["colors"]), gref["colors"])
    _say(f"[variant] {label} v{variant}: {eg}")
    assert_grads(eg, f"{label} variant {variant}")


@pytest.mark.parametrize("variant", range(9))
@pytest.mark.parametrize("label,n,views", VARIANT_CASES, ids=[c[0] for c in VARIANT_CASES])
def test_backward_variants_without_normals(fmb, variant, label, n, views):
    """Every backward variant (Gaussian-lane 0-2, ray-lane 3-5, tiled 6-8) takes the offset form of
    the adjoint without a normal cotangent: against the oracle with depth, alpha, two-way flow and
    colour cotangents."""
    sc, cams = custom_scene(n, views, seed=310 + n, flow=True)
    cams = W.with_backward_flow(cams, seed=311)
    g = np.random.Generator(np.random.PCG64(312))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    _say(f"[variant-plain] {label} bwd variant {variant}: N={n} views={views}")
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    fmb.set_launch_config(scene=scene, bwd_variant=variant)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    scene.set_colors(t(q))
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, betas, 1.0, colors=q)
    hit = ref["alpha"] >= 1e-3
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 313, flow=False), ref["alpha"])
    cot["normal"] = None
    cot["flow"] = (g.standard_normal((cams.n_rays, 4)) * hit[:, None]).astype(np.float32)
    cot["color"] = (g.standard_normal((cams.n_rays, 3)) * hit[:, None]).astype(np.float32)
    gr = scene.backward(outs, t(cot["depth"]), t(cot["alpha"]), None, t(cot["flow"]), g_color=t(cot["color"]))
    torch.cuda.synchronize()
    assert fmb.launch_config(scene=scene)["bwd_variant"] == variant
    _, gref, _ = O.render_workload_view(sc, cams, betas, 1.0, cot=cot, colors=q)
    eg = compare_grads(gr, gref)
    eg["colors"] = normwise(to_np(gr["colors"]), gref["colors"])
    _say(f"[variant-plain] {label} v{variant}: {eg}")
    assert_grads(eg, f"{label} variant {variant} without normals")


@pytest.mark.parametrize("variant", range(4))
def test_forward_variants(fmb, variant):
    """Every forward tile variant (rays per lane 1, 2, 4; tile 128 or 256 Gaussians) against the
    oracle on ragged views, with normals, two-way flow and colour."""
    sc, cams = custom_scene(257, [(40, 50), (3, 7), (1, 1)], seed=400, flow=True)
    cams = W.with_backward_flow(cams, seed=401)
    g = np.random.Generator(np.random.PCG64(402))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    _say(f"[fwd-variant] {variant}: N={sc.n} P={cams.n_rays}")
    scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
    fmb.set_launch_config(scene=scene, fwd_variant=variant)
    scene.set_colors(torch.as_tensor(q, device=DEV).contiguous())
    outs = scene.render(normals=True)
    torch.cuda.synchronize()
    assert fmb.launch_config(scene=scene)["fwd_variant"] == variant
    ref, _, _ = O.render_workload_view(sc, cams, betas, 1.0, colors=q)
    e = compare_forward(outs, ref)
    e["color"] = normwise(to_np(outs["color"]), ref["color"])
    _say(f"[fwd-variant] {variant}: {e}")
    assert_forward(e, f"forward variant {variant}")
    assert e["color"] <= TOL_REL


# ---------------------------------------------------------------------------------------
# The benchmarked steps of the large and the two-way-flow workloads: cotangents of the
# reconstruction loss (Sec. 4) only, no normal cotangent, so every backward variant takes the
# short (A, Bv, L) adjoint.  The cotangents are the oracle's loss gradient on a seeded sample
# of rays (targets rendered by the oracle from the perturbed scene) and zero elsewhere, so the
# oracle's gradient over the sample is the exact reference for the GPU gradient over the image.
# ---------------------------------------------------------------------------------------

def _loss_step_setup(fmb, name, k, seed, two_way=False):
    w = W.make_config(name)
    sc, cams = w.scenes[0], w.cameras[0]
    if two_way:
        cams = W.with_backward_flow(cams, seed=11)
    p = cams.n_rays
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    outs = scene.render(normals=w.normals, flow=cams.has_flow)
    rays = _sample(p, k, seed)
    ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays)
    tgt, _, _ = O.render_workload_view(w.targets[0], cams, w.betas, w.eta, rays=rays)
    flow = ref.get("flow") if cams.has_flow else None
    _, lg = O.loss_grad(ref["depth"], ref["alpha"], tgt["depth"], tgt["alpha"], flow,
                        tgt.get("flow") if flow is not None else None, 1.0, 0.1, 2)
    cs = {"depth": lg["depth"].astype(np.float32), "alpha": lg["alpha"].astype(np.float32), "normal": None,
          "flow": None if flow is None else lg["flow"].astype(np.float32)}
    _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays, cot=cs)
    cot = {"normal": None, "flow": None}
    for key in ("depth", "alpha", "flow"):
        if cs[key] is not None:
            full = np.zeros((p,) + cs[key].shape[1:], np.float32)
            full[rays] = cs[key]
            cot[key] = torch.as_tensor(full, device=DEV).contiguous()
    torch.cuda.synchronize()
    return scene, outs, cot, gref


LOSS_STEPS = [("large1080", 2000, 13, False), ("flow480", 20000, 17, True)]


@pytest.fixture(scope="module", params=LOSS_STEPS, ids=[c[0] for c in LOSS_STEPS])
def loss_step(fmb, request):
    name, k, seed, two_way = request.param
    _say(f"[loss-step] {name}: oracle loss gradient on {k} sampled rays")
    return (name,) + _loss_step_setup(fmb, name, k, seed, two_way)


@pytest.mark.parametrize("variant", list(range(9)) + ["tuned"])
def test_loss_step_backward_variants(fmb, loss_step, variant):
    name, scene, outs, cot, gref = loss_step
    grads = scene.backward(outs, cot["depth"], cot["alpha"], None, cot["flow"])
    if variant == "tuned":
        scene.autotune(outs, cot, grads)
        scene.render(normals=outs.get("normal") is not None, flow=cot["flow"] is not None, out=outs)
    else:
        fmb.set_launch_config(scene=scene, fwd_variant=fmb.launch_config(scene=scene)["fwd_variant"],
                              bwd_variant=variant)
    g = scene.backward(outs, cot["depth"], cot["alpha"], None, cot["flow"], grads=grads)
    torch.cuda.synchronize()
    e = compare_grads(g, gref)
    _say(f"[loss-step] {name} backward variant {variant} ({fmb.launch_config(scene=scene)}): {fmt(e)}")
    assert_grads(e, f"{name} loss step, backward variant {variant}")
