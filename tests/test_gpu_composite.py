"""GPU parity of the zero-parameter renderer (alpha compositing, Eq. 9-10) against the oracle.

Every case renders through the C ABI with the compositing model selected and compares with
the FP64 oracle's compositing model on the same seeded inputs: scene sizes from one Gaussian to
scenes staged in several LDS tiles (N = 1 ... 600), clustered scenes whose tiles need several
depth windows, the 10 000-Gaussian 1080p scene on sampled rays, ragged images, tied
intersections, Gaussians behind the camera, colours and both flow directions, the batched path,
and the gradient of the workload loss.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import (TOL_REL, assert_forward, assert_grads, compare_forward, compare_grads,
                            custom_scene, hit_mask_cot, make_scene, normwise, to_np)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
BETAS = np.array([W.BETA1, W.BETA2], np.float32)


@pytest.fixture(scope="module")
def fmb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_14737_amd as m
    return m


def _say(*a):
    print(*a, flush=True)


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()


def _composite_scene(fmb, sc, cams):
    scene, params = make_scene(fmb, torch, sc, cams, BETAS, 1.0, DEV)
    scene.set_model("composite")
    return scene, params


CASES = [
    ("n1_odd", 1, [(17, 23)]),
    ("n7_multi", 7, [(5, 3), (64, 64), (1, 1), (33, 65)]),
    ("n40", 40, [(48, 64), (31, 17)]),
    ("n64_full_wave", 64, [(40, 50)]),
    ("n100_two_per_lane", 100, [(40, 50), (3, 7)]),
    ("n256_four_per_lane", 256, [(24, 32)]),
]


@pytest.mark.parametrize("label,n,views", CASES, ids=[c[0] for c in CASES])
def test_composite_parity(fmb, label, n, views):
    sc, cams = custom_scene(n, views, seed=100 + n, flow=True)
    _say(f"[composite] {label}: N={n} views={views}")
    scene, _ = _composite_scene(fmb, sc, cams)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, BETAS, 1.0, model="composite")
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 6, flow=True), ref["alpha"])
    g = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), _t(cot["normal"]), _t(cot["flow"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, model="composite")
    e = compare_forward(outs, ref)
    eg = compare_grads(g, gref)
    _say(f"[composite] {label}: {e} {eg}")
    assert_forward(e, label)
    assert_grads(eg, label)
    assert torch.count_nonzero(g["betas"]).item() == 0


@pytest.mark.parametrize("label,n,views", [CASES[1], CASES[4], CASES[5]], ids=[CASES[i][0] for i in (1, 4, 5)])
def test_composite_parity_without_normals(fmb, label, n, views):
    """Without a normal cotangent the compositing adjoint takes the (A, Bv, L) form; depth, alpha,
    two-way flow cotangents against the oracle, at two and four Gaussians per lane."""
    sc, cams = custom_scene(n, views, seed=120 + n, flow=True)
    _say(f"[composite-plain] {label}: N={n} views={views}")
    scene, _ = _composite_scene(fmb, sc, cams)
    outs = scene.render(normals=False)
    ref, _, _ = O.render_workload_view(sc, cams, BETAS, 1.0, model="composite")
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 8, flow=True, normals=False), ref["alpha"])
    g = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), None, _t(cot["flow"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, model="composite")
    eg = compare_grads(g, gref)
    _say(f"[composite-plain] {label}: {eg}")
    assert_grads(eg, label)


@pytest.mark.parametrize("label,n,views", [CASES[1], CASES[2], CASES[4], CASES[5]],
                         ids=[CASES[i][0] for i in (1, 2, 4, 5)])
def test_composite_colour_without_normals(fmb, label, n, views):
    """A colour cotangent without a normal cotangent: the slots' z_bar takes the colour term of
    their Gaussians (C_bar . c), with depth, alpha and two-way flow cotangents, against the oracle."""
    sc, cams = custom_scene(n, views, seed=140 + n, flow=True)
    cams = W.with_backward_flow(cams, seed=141)
    g = np.random.Generator(np.random.PCG64(142))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    _say(f"[composite-colour-plain] {label}: N={n} views={views}")
    scene, _ = _composite_scene(fmb, sc, cams)
    scene.set_colors(_t(q))
    outs = scene.render(normals=False)
    ref, _, _ = O.render_workload_view(sc, cams, BETAS, 1.0, colors=q, model="composite")
    hit = ref["alpha"] >= 1e-3
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 143, flow=False, normals=False), ref["alpha"])
    cot["flow"] = (g.standard_normal((cams.n_rays, 4)) * hit[:, None]).astype(np.float32)
    cot["color"] = (g.standard_normal((cams.n_rays, 3)) * hit[:, None]).astype(np.float32)
    gr = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), None, _t(cot["flow"]), g_color=_t(cot["color"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, colors=q, model="composite")
    eg = compare_grads(gr, gref)
    eg["colors"] = normwise(to_np(gr["colors"]), gref["colors"])
    _say(f"[composite-colour-plain] {label}: {eg}")
    assert_grads(eg, label)


def test_composite_ties_and_behind(fmb):
    """Copies of the same Gaussian (equal t on every ray: no mutual attenuation) and Gaussians
    behind the front camera."""
    sc, cams = custom_scene(30, [(40, 48), (17, 9)], seed=7, behind=True)
    dup = np.array([3, 3, 3, 11, 11])
    sc = W.Scene(np.concatenate([sc.means, sc.means[dup]]), np.concatenate([sc.prec, sc.prec[dup]]),
                 np.concatenate([sc.weights, sc.weights[dup]]))
    _say(f"[composite-ties] N={sc.n} P={cams.n_rays}")
    scene, _ = _composite_scene(fmb, sc, cams)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, BETAS, 1.0, model="composite")
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 8, flow=False), ref["alpha"])
    g = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), _t(cot["normal"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, model="composite")
    e, eg = compare_forward(outs, ref), compare_grads(g, gref)
    _say(f"[composite-ties] {e} {eg}")
    # Gaussians behind the camera: per pixel the blended depth can cancel to near zero (norm-wise only)
    assert_forward(e, "ties", per_pixel=False)
    assert_grads(eg, "ties")


def test_composite_colour_two_way_flow_quality(fmb):
    """Colours, forward and backward flow, and the quality value max_i w_i (from the stash)."""
    sc, cams = custom_scene(50, [(36, 44), (20, 30)], seed=9, flow=True)
    cams = W.with_backward_flow(cams, seed=10)
    g = np.random.Generator(np.random.PCG64(11))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    _say(f"[composite-colour] N={sc.n} P={cams.n_rays}")
    scene, _ = _composite_scene(fmb, sc, cams)
    scene.set_colors(_t(q))
    outs = scene.render(normals=True)
    ref, _, (view, row, col) = O.render_workload_view(sc, cams, BETAS, 1.0, colors=q, model="composite")
    e = compare_forward(outs, ref)
    e["color"] = normwise(to_np(outs["color"]), ref["color"])
    hit = ref["alpha"] >= 1e-3
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 12, flow=False), ref["alpha"])
    cot["flow"] = (g.standard_normal((cams.n_rays, 4)) * hit[:, None]).astype(np.float32)
    cot["color"] = (g.standard_normal((cams.n_rays, 3)) * hit[:, None]).astype(np.float32)
    gr = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), _t(cot["normal"]), _t(cot["flow"]),
                        g_color=_t(cot["color"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, colors=q, model="composite")
    eg = compare_grads(gr, gref)
    eg["colors"] = normwise(to_np(gr["colors"]), gref["colors"])
    rs = np.flatnonzero(hit)[:: max(1, int(hit.sum()) // 300)]
    o, v = O.pixel_rays(view[rs], row[rs], col[rs], cams.w2c, cams.intr)
    osc = O.OracleScene.of(sc.means, sc.prec, sc.weights, BETAS, 1.0)
    e["quality"] = float(np.max(np.abs(to_np(fmb.Scene.quality(outs))[rs]
                                       - O.max_weight(osc, o, v, model="composite"))))
    _say(f"[composite-colour] {e} {eg}")
    assert_forward(e, "colour")
    assert e["color"] <= TOL_REL and e["quality"] <= TOL_REL
    assert_grads(eg, "colour")


def test_composite_loss_gradient_fwdbwd128(fmb):
    """The fwdbwd128 workload (N = 40, 20 views of 128 x 128) with the compositing model: every
    ray's forward outputs, and the gradient of the workload loss (alpha-weighted L1 depth + BCE
    alpha against targets rendered from the perturbed scene by the oracle)."""
    w = W.make_config("fwdbwd128")
    sc, cams = w.scenes[0], w.cameras[0]
    _say("[composite-loss] fwdbwd128")
    scene, _ = _composite_scene(fmb, sc, cams)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta, model="composite")
    tgt, _, _ = O.render_workload_view(w.targets[0], cams, w.betas, w.eta, model="composite")
    p = cams.n_rays
    gd = tgt["alpha"] * np.sign(ref["depth"] - tgt["depth"]) / p
    a = np.clip(ref["alpha"], 1e-6, 1 - 1e-6)
    inside = (ref["alpha"] >= 1e-6) & (ref["alpha"] <= 1 - 1e-6)
    ga = np.where(inside, (a - tgt["alpha"]) / (a * (1 - a)), 0.0) / p
    cot = {"depth": gd.astype(np.float32), "alpha": ga.astype(np.float32), "normal": None, "flow": None}
    g = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, cot=cot, model="composite")
    e, eg = compare_forward(outs, ref), compare_grads(g, gref)
    _say(f"[composite-loss] {e} {eg}")
    assert_forward(e, "fwdbwd128 composite")
    assert_grads(eg, "fwdbwd128 composite loss")


def test_composite_batch(fmb):
    """Batched compositing: every scene of a batch matches its single-scene render bit for bit
    (items never span scenes), and the batch matches the oracle."""
    w = W.make_config("batch16")
    for idx in ([2, 8, 10], [1, 12, 3]):
        scenes = [w.scenes[i] for i in idx]
        camsl = [w.cameras[i] for i in idx]
        ns = [s.n for s in scenes]
        means = _t(np.concatenate([s.means for s in scenes]))
        prec = _t(np.concatenate([s.prec for s in scenes]))
        weights = _t(np.concatenate([s.weights for s in scenes]))
        betas = _t(np.tile(w.betas, (len(scenes), 1)))
        cams = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, device=DEV) for c in camsl]
        b = fmb.Batch(means, prec, weights, betas, [w.eta] * len(scenes), ns, cams)
        b.set_model("composite")
        _say(f"[composite-batch] scenes {idx} N={ns} P={b.n_rays}")
        outs = b.forward(b.alloc_outputs(normals=True))
        gc = W.random_cotangents(b.n_rays, 21, flow=False)
        cot = {"depth": _t(gc["depth"]), "alpha": _t(gc["alpha"]), "normal": _t(gc["normal"]), "flow": None}
        grads = b.backward(outs, cot, b.alloc_grads())
        torch.cuda.synchronize()
        for i in range(len(scenes)):
            r0, r1 = b.ray_off[i], b.ray_off[i + 1]
            g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
            scene = fmb.Scene(means[g0:g1], prec[g0:g1], weights[g0:g1], betas[i], w.eta, cams[i])
            scene.set_model("composite")
            so = scene.render(normals=True)
            sg = scene.backward(so, cot["depth"][r0:r1], cot["alpha"][r0:r1], cot["normal"][r0:r1])
            torch.cuda.synchronize()
            for k in ("depth", "alpha", "normal", "stash"):
                assert torch.equal(outs[k][r0:r1], so[k]), (idx, i, k)
            for k in ("means", "prec", "weights"):
                assert torch.equal(grads[k][g0:g1], sg[k]), (idx, i, k)
            ref, _, _ = O.render_workload_view(scenes[i], camsl[i], w.betas, w.eta, model="composite")
            e = compare_forward({k: v[r0:r1] if v is not None else None for k, v in outs.items()}, ref)
            _say(f"[composite-batch] scene {idx[i]} N={ns[i]} {e}")
            assert_forward(e, f"batch scene {idx[i]}")


def test_composite_model_switch(fmb):
    """Switching a scene between the two models gives each model's own result, and the
    compositing model takes scenes of any size (here 257 Gaussians, two LDS tiles)."""
    sc, cams = custom_scene(20, [(16, 16)], seed=3)
    scene, _ = make_scene(fmb, torch, sc, cams, BETAS, 1.0, DEV)
    blend1 = scene.render(normals=False)["depth"].clone()
    scene.set_model("composite")
    comp = scene.render(normals=False)["depth"].clone()
    scene.set_model("blend")
    blend2 = scene.render(normals=False)["depth"].clone()
    torch.cuda.synchronize()
    assert torch.equal(blend1, blend2)
    assert not torch.equal(blend1, comp)
    big, bcams = custom_scene(257, [(4, 4)], seed=4)
    bscene, _ = _composite_scene(fmb, big, bcams)
    outs = bscene.render(normals=True)
    torch.cuda.synchronize()
    ref, _, _ = O.render_workload_view(big, bcams, BETAS, 1.0, model="composite")
    e = compare_forward(outs, ref)
    _say(f"[composite-switch] N=257 {e}")
    assert_forward(e, "N=257 after the switch")


def _cluster_scene(n, views, seed, spread):
    """n Gaussians clustered around the origin (normal, standard deviation `spread`): the rays
    through the centre pass all of them at significant densities, so their tiles take several
    depth windows of the compositing kernels."""
    _, cams = custom_scene(1, views, seed)
    g = np.random.Generator(np.random.PCG64(seed + 1))
    return W.make_scene(g, n, g.normal(0.0, spread, (n, 3))), cams


WINDOWS = [
    ("n90_resident", 90, [(24, 24)], 0.05),
    ("n300_staged", 300, [(16, 20), (9, 7)], 0.08),
    ("n600_staged", 600, [(12, 12)], 0.1),
]


@pytest.mark.parametrize("label,n,views,spread", WINDOWS, ids=[c[0] for c in WINDOWS])
def test_composite_depth_windows(fmb, label, n, views, spread):
    """Scenes whose central tiles have more significant intersections than the kernels' slots:
    forward and gradients over several depth windows match the oracle."""
    sc, cams = _cluster_scene(n, views, seed=n, spread=spread)
    _say(f"[composite-windows] {label}: N={n} views={views}")
    scene, _ = _composite_scene(fmb, sc, cams)
    outs = scene.render(normals=True)
    ref, _, _ = O.render_workload_view(sc, cams, BETAS, 1.0, model="composite")
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 9, flow=False), ref["alpha"])
    g = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), _t(cot["normal"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, model="composite")
    e = compare_forward(outs, ref)
    eg = compare_grads(g, gref)
    _say(f"[composite-windows] {label}: {e} {eg}")
    assert_forward(e, label)
    assert_grads(eg, label)
    # the plain adjoint (depth and alpha cotangents) over the same windows
    cot2 = dict(cot, normal=None)
    g2 = scene.backward(outs, _t(cot2["depth"]), _t(cot2["alpha"]), None)
    torch.cuda.synchronize()
    _, gref2, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot2, model="composite")
    eg2 = compare_grads(g2, gref2)
    _say(f"[composite-windows] {label} plain: {eg2}")
    assert_grads(eg2, label + " plain")


def test_composite_colour_windows_without_normals(fmb):
    """Colour and depth/alpha cotangents without a normal cotangent on a clustered scene staged
    through LDS whose central tiles take several depth windows, against the oracle."""
    label, n, views, spread = WINDOWS[1]
    sc, cams = _cluster_scene(n, views, seed=n + 7, spread=spread)
    g = np.random.Generator(np.random.PCG64(144))
    q = (1.5 * g.standard_normal((sc.n, 3))).astype(np.float32)
    _say(f"[composite-colour-windows] {label}: N={n} views={views}")
    scene, _ = _composite_scene(fmb, sc, cams)
    scene.set_colors(_t(q))
    outs = scene.render(normals=False)
    ref, _, _ = O.render_workload_view(sc, cams, BETAS, 1.0, colors=q, model="composite")
    hit = ref["alpha"] >= 1e-3
    cot = hit_mask_cot(W.random_cotangents(cams.n_rays, 145, flow=False, normals=False), ref["alpha"])
    cot["color"] = (g.standard_normal((cams.n_rays, 3)) * hit[:, None]).astype(np.float32)
    gr = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), None, None, g_color=_t(cot["color"]))
    torch.cuda.synchronize()
    _, gref, _ = O.render_workload_view(sc, cams, BETAS, 1.0, cot=cot, colors=q, model="composite")
    e = compare_forward(outs, ref)
    e["color"] = normwise(to_np(outs["color"]), ref["color"])
    eg = compare_grads(gr, gref)
    eg["colors"] = normwise(to_np(gr["colors"]), gref["colors"])
    _say(f"[composite-colour-windows] {label}: {e} {eg}")
    assert_forward(e, label)
    assert e["color"] <= TOL_REL
    assert_grads(eg, label)


def _hit_sample(alpha, k, seed):
    """k ray indices, half of them among the rays that see the scene (alpha >= 0.01)."""
    g = np.random.Generator(np.random.PCG64(seed))
    hit = np.flatnonzero(alpha >= 0.01)
    a = g.choice(hit, size=min(k // 2, hit.size), replace=False)
    b = g.choice(alpha.size, size=k - a.size, replace=False)
    return np.unique(np.concatenate([a, b]))


def test_composite_large1080(fmb):
    """The 10 000-Gaussian 1080p scene with the compositing model: the forward on sampled rays
    (half of them on the object, where the tiles take several depth windows) and the gradient of
    random cotangents on a smaller sample, against the oracle on those rays."""
    w = W.make_config("large1080")
    sc, cams = w.scenes[0], w.cameras[0]
    p = cams.n_rays
    _say(f"[composite-large1080] N={sc.n} P={p}")
    scene, _ = _composite_scene(fmb, sc, cams)
    outs = scene.render(normals=True)
    torch.cuda.synchronize()
    alpha = to_np(outs["alpha"])
    rays = _hit_sample(alpha, 96, 5)
    ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays, model="composite")
    e = compare_forward(outs, ref, rays)
    _say(f"[composite-large1080] forward on {rays.size} rays: {e}")
    assert_forward(e, "large1080 composite")
    brays = rays[::3]
    cot = W.random_cotangents(p, 77, flow=False, normals=False)
    mask = np.zeros(p, dtype=bool)
    mask[brays] = True
    for k in ("depth", "alpha"):
        cot[k][~mask] = 0.0
    g = scene.backward(outs, _t(cot["depth"]), _t(cot["alpha"]), None)
    torch.cuda.synchronize()
    cot_s = {"depth": cot["depth"][brays], "alpha": cot["alpha"][brays], "normal": None, "flow": None}
    _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=brays, cot=cot_s, model="composite")
    eg = compare_grads(g, gref)
    _say(f"[composite-large1080] gradient of {brays.size} rays: {eg}")
    assert_grads(eg, "large1080 composite gradient")


def test_composite_graph_replay(fmb):
    """The compositing passes captured in HIP graphs replay like the eager calls, several times
    with eager work in between, and see in-place parameter updates."""
    w = W.make_config("batch16")
    idx = [2, 5, 9]
    scenes = [w.scenes[i] for i in idx]
    means = _t(np.concatenate([s.means for s in scenes]))
    prec = _t(np.concatenate([s.prec for s in scenes]))
    weights = _t(np.concatenate([s.weights for s in scenes]))
    betas = _t(np.tile(w.betas, (len(scenes), 1)))
    cams = [fmb.Cameras.from_numpy(w.cameras[i].w2c, w.cameras[i].intr, w.cameras[i].hw, device=DEV) for i in idx]
    b = fmb.Batch(means, prec, weights, betas, [w.eta] * len(scenes), [s.n for s in scenes], cams)
    b.set_model("composite")
    gc = W.random_cotangents(b.n_rays, 55, flow=False)
    cot = {"depth": _t(gc["depth"]), "alpha": _t(gc["alpha"]), "normal": _t(gc["normal"]), "flow": None}
    outs_g, grads_g = b.alloc_outputs(normals=True), b.alloc_grads()
    outs_e, grads_e = b.alloc_outputs(normals=True), b.alloc_grads()
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    _say(f"[composite-graph] scenes {idx} P={b.n_rays}")
    b.capture(outs_g, cot, grads_g, st)
    for rep in range(3):
        with torch.cuda.stream(st):
            b.graph_launch(2, st)
        st.synchronize()
        b.forward(outs_e)
        b.backward(outs_e, cot, grads_e)
        torch.cuda.synchronize()
        for k in ("depth", "alpha", "normal", "stash"):
            assert torch.equal(outs_g[k], outs_e[k]), (rep, k)
        for k in ("means", "prec", "weights", "betas"):
            assert torch.equal(grads_g[k], grads_e[k]), (rep, k)
        with torch.no_grad():
            means.add_(0.001)
