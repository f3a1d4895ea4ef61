"""GPU tests of the batched persistent form and its HIP-graph capture."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import (TOL_REL, assert_forward, assert_grads, compare_forward, compare_grads, fmt,
                            make_scene, normwise, to_np)

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


def _batch_inputs(w, fmb):
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    means = t(np.concatenate([s.means for s in w.scenes]))
    prec = t(np.concatenate([s.prec for s in w.scenes]))
    weights = t(np.concatenate([s.weights for s in w.scenes]))
    betas = t(np.tile(w.betas, (len(w.scenes), 1)))
    cams = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, c.w2c_b, c.intr_b, device=DEV) for c in w.cameras]
    b = fmb.Batch(means, prec, weights, betas, [w.eta] * len(w.scenes), [s.n for s in w.scenes], cams)
    return b, (means, prec, weights, betas)


def _cotangents(b, seed, normals=True):
    cot = W.random_cotangents(b.n_rays, seed, flow=b.has_flow, normals=normals)
    return {k: (None if v is None else torch.as_tensor(v, device=DEV).contiguous()) for k, v in cot.items()}


@pytest.fixture(scope="module")
def batch16(fmb):
    w = W.make_config("batch16")
    b, params = _batch_inputs(w, fmb)
    return w, b, params


def test_batch_equals_plain_bitwise(fmb, batch16):
    """The persistent batched kernels and per-scene plain launches cut each scene into the
    same items, so outputs and gradients agree bit for bit."""
    w, b, params = batch16
    _say(f"[batch] batch16 S={len(w.scenes)} P={b.n_rays} pairs={w.n_pairs}")
    outs = b.forward(b.alloc_outputs(normals=True))
    cot = _cotangents(b, 21)
    grads = b.backward(outs, cot, b.alloc_grads())
    torch.cuda.synchronize()
    for i, (sc, cams) in enumerate(zip(w.scenes, w.cameras)):
        scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        o = scene.render(normals=True)
        gi = scene.backward(o, cot["depth"][r0:r1], cot["alpha"][r0:r1],
                            None if cot["normal"] is None else cot["normal"][r0:r1])
        torch.cuda.synchronize()
        for k in ("depth", "alpha", "normal", "stash"):
            assert torch.equal(o[k], outs[k][r0:r1]), (i, k)
        for k in ("means", "prec", "weights"):
            assert torch.equal(gi[k], grads[k][g0:g1]), (i, k)
        assert torch.equal(gi["betas"], grads["betas"][i]), (i, "betas")


def test_batch_vs_oracle(fmb, batch16):
    """Every scene of the batch against the oracle: sampled rays forward, and one backward with
    seeded cotangents on sampled rays of every scene (zero elsewhere), whose gradient over each
    scene is compared with the oracle's over that scene's sample."""
    w, b, params = batch16
    outs = b.forward(b.alloc_outputs(normals=True))
    cot = W.random_cotangents(b.n_rays, 33, flow=False)
    g = np.random.Generator(np.random.PCG64(5))
    samples = []
    for i, (sc, cams) in enumerate(zip(w.scenes, w.cameras)):
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        samples.append(np.sort(g.choice(r1 - r0, size=min(1500, r1 - r0), replace=False)))
    full = {k: np.zeros_like(v) for k, v in cot.items() if v is not None}
    for i, rays in enumerate(samples):
        for k in full:
            full[k][b.ray_off[i] + rays] = cot[k][b.ray_off[i] + rays]
    tc = {k: torch.as_tensor(v, device=DEV).contiguous() for k, v in full.items()}
    grads = b.backward(outs, tc, b.alloc_grads())
    torch.cuda.synchronize()
    for i, (sc, cams) in enumerate(zip(w.scenes, w.cameras)):
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        rays = samples[i]
        cs = {k: v[r0 + rays] for k, v in full.items()}
        cs["flow"] = None
        ref, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays, cot=cs)
        sub = {k: (None if v is None else v[r0:r1]) for k, v in outs.items()}
        e = compare_forward(sub, ref, rays)
        gs = {"means": grads["means"][g0:g1], "prec": grads["prec"][g0:g1], "weights": grads["weights"][g0:g1],
              "betas": grads["betas"][i]}
        eg = compare_grads(gs, gref)
        _say(f"[batch-oracle] scene {i} N={sc.n} V={cams.v} {cams.hw[0]}: {fmt(e)} {fmt(eg)}")
        assert_forward(e, f"scene {i}")
        assert_grads(eg, f"batch scene {i}")


def test_graph_replay(fmb, batch16):
    """A captured forward+backward replays like the eager batched calls, several times with eager
    work in between, and sees in-place parameter updates."""
    w, b, (means, prec, weights, betas) = batch16
    outs_e = b.alloc_outputs(normals=True)
    grads_e = b.alloc_grads()
    cot = _cotangents(b, 44)
    outs_g = b.alloc_outputs(normals=True)
    grads_g = b.alloc_grads()
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    _say("[graph] capture")
    b.capture(outs_g, cot, grads_g, st)
    for rep in range(3):
        with torch.cuda.stream(st):
            b.graph_launch(2, st)
        st.synchronize()
        b.forward(outs_e)
        b.backward(outs_e, cot, grads_e)
        torch.cuda.synchronize()
        for k in ("depth", "alpha", "normal"):
            assert torch.equal(outs_g[k], outs_e[k]), (rep, k)
        for k in grads_e:
            if grads_e[k] is not None:
                assert torch.equal(grads_g[k], grads_e[k]), (rep, k)
        _say(f"[graph] replay {rep} matches eager")
        # in-place update seen by the next replay
        with torch.no_grad():
            means.add_(0.001)
            betas.mul_(1.01)


@pytest.mark.parametrize("model", ["blend", "composite"])
def test_forward_loss_fused(fmb, batch16, model):
    """The forward with the loss's depth and alpha cotangents written in its epilogue equals the
    forward followed by the loss kernel, outputs and cotangents bit for bit."""
    w, b, _ = batch16
    b.set_model(model)
    try:
        g = np.random.Generator(np.random.PCG64(46))
        d_t = torch.as_tensor(3.0 + g.random(b.n_rays).astype(np.float32), device=DEV)
        a_t = torch.as_tensor((g.random(b.n_rays) > 0.5).astype(np.float32), device=DEV)
        _say(f"[fused-loss] {model}")
        outs1 = b.forward(b.alloc_outputs(normals=True))
        ref = fmb.loss_grad(outs1, d_t, a_t, w_depth=0.7)
        outs2 = b.alloc_outputs(normals=True)
        cot = {"depth": torch.full((b.n_rays,), float("nan"), device=DEV),
               "alpha": torch.full((b.n_rays,), float("nan"), device=DEV)}
        b.forward_loss(outs2, d_t, a_t, cot, w_depth=0.7)
        torch.cuda.synchronize()
        for k in ("depth", "alpha", "normal", "stash"):
            assert torch.equal(outs1[k], outs2[k]), k
        assert torch.equal(cot["depth"], ref["depth"])
        assert torch.equal(cot["alpha"], ref["alpha"])
    finally:
        b.set_model("blend")


def test_whole_step_single_graph(fmb, batch16):
    """The whole training step — forward, the loss kernel's cotangents, backward, finalize — captured
    from its stream as ONE graph replays like the eager calls, several times with eager work in
    between (the library calls allocate nothing and record no memset)."""
    w, b, _ = batch16
    outs = b.alloc_outputs(normals=True)
    grads = b.alloc_grads()
    g = np.random.Generator(np.random.PCG64(45))
    d_t = torch.as_tensor(3.0 + g.random(b.n_rays).astype(np.float32), device=DEV)
    a_t = torch.as_tensor((g.random(b.n_rays) > 0.5).astype(np.float32), device=DEV)
    cot = {"depth": torch.empty(b.n_rays, device=DEV), "alpha": torch.empty(b.n_rays, device=DEV),
           "normal": None, "flow": None}

    def step():
        b.forward(outs)
        fmb.loss_grad(outs, d_t, a_t, cot=cot)
        b.backward(outs, cot, grads)

    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        step()
    torch.cuda.current_stream().wait_stream(s2)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in grads.items() if v is not None}
    graph = torch.cuda.CUDAGraph()
    _say("[step-graph] capture")
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        for v in grads.values():
            if v is not None:
                v.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        for k, v in ref.items():
            assert torch.equal(grads[k], v), (rep, k)
        step()  # eager work between replays
        torch.cuda.synchronize()
        _say(f"[step-graph] replay {rep} matches eager")


@pytest.mark.parametrize("variant", [3, 5, 6, 7, 8])
def test_ray_lane_batch_bitwise(fmb, batch16, variant):
    """The ray-lane backward kernels, batched and persistent, equal per-scene plain launches of
    the same variant bit for bit (items are cut per scene); the tiled variants 6-8 without a
    normal cotangent (which they hand to variant 2)."""
    w, b, params = batch16
    fmb.set_launch_config(batch=b, bwd_variant=variant)
    _say(f"[ray-lane] batch16 bwd variant {variant}")
    outs = b.forward(b.alloc_outputs(normals=True))
    cot = _cotangents(b, 23, normals=variant < 6)
    grads = b.backward(outs, cot, b.alloc_grads())
    torch.cuda.synchronize()
    means, prec, weights, betas = params  # the batch's current parameters (other tests update them)
    for i in (0, 6, 8, 12):
        cams = w.cameras[i]
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        scene = fmb.Scene(means[g0:g1], prec[g0:g1], weights[g0:g1], betas[i], w.eta,
                          fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, cams.w2c_b, cams.intr_b, device=DEV))
        fmb.set_launch_config(scene=scene, bwd_variant=variant)
        o = scene.render(normals=True)
        gi = scene.backward(o, cot["depth"][r0:r1], cot["alpha"][r0:r1],
                            None if cot["normal"] is None else cot["normal"][r0:r1])
        torch.cuda.synchronize()
        for k in ("means", "prec", "weights"):
            assert torch.equal(gi[k], grads[k][g0:g1]), (i, k)
        assert torch.equal(gi["betas"], grads["betas"][i]), (i, "betas")
    fmb.set_launch_config(batch=b)


def test_bench_configuration(fmb, batch16):
    """The benchmark's own configuration: the autotuned persistent kernels on batch16, tuned with
    the loss kernel's cotangents.  Forward outputs of every scene on sampled rays against the
    oracle; then one backward whose cotangents are the oracle's gradient of the workload loss
    (alpha-weighted L1 depth + BCE alpha against the oracle's render of the perturbed scene) on
    sampled rays of every scene, zero elsewhere, against the oracle's gradient per scene."""
    w, b, (means, prec, weights, betas) = batch16
    outs = b.alloc_outputs(normals=True)
    grads = b.alloc_grads()
    g = np.random.Generator(np.random.PCG64(91))
    d_t = torch.as_tensor(g.uniform(1.0, 5.0, b.n_rays).astype(np.float32), device=DEV)
    a_t = torch.as_tensor((g.uniform(0, 1, b.n_rays) > 0.5).astype(np.float32), device=DEV)
    cot = {"depth": torch.empty(b.n_rays, device=DEV), "alpha": torch.empty(b.n_rays, device=DEV),
           "normal": None, "flow": None}
    b.forward(outs)
    fmb.loss_grad(outs, d_t, a_t, cot=cot)
    b.backward(outs, cot, grads)
    b.autotune(outs, cot, grads)
    cfg = fmb.launch_config(batch=b)
    _say(f"[bench-config] {cfg}")
    b.forward(outs)
    torch.cuda.synchronize()
    sc_means = to_np(means).astype(np.float32)
    sc_prec = to_np(prec).astype(np.float32)
    sc_weights = to_np(weights).astype(np.float32)
    full = {k: np.zeros(b.n_rays, np.float32) for k in ("depth", "alpha")}
    per_scene = []
    for i, cams in enumerate(w.cameras):
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        sc = W.Scene(sc_means[g0:g1], sc_prec[g0:g1], sc_weights[g0:g1])
        bi = to_np(betas[i]).astype(np.float32)
        rays = np.sort(g.choice(r1 - r0, size=min(1500, r1 - r0), replace=False))
        ref, _, _ = O.render_workload_view(sc, cams, bi, w.eta, rays=rays)
        sub = {k: (None if v is None else v[r0:r1]) for k, v in outs.items()}
        e = compare_forward(sub, ref, rays)
        _say(f"[bench-config] scene {i} forward {fmt(e)}")
        assert_forward(e, f"bench configuration scene {i}")
        tgt, _, _ = O.render_workload_view(w.targets[i], cams, bi, w.eta, rays=rays)
        _, lg = O.loss_grad(ref["depth"], ref["alpha"], tgt["depth"], tgt["alpha"])
        cs = {"depth": lg["depth"].astype(np.float32), "alpha": lg["alpha"].astype(np.float32),
              "normal": None, "flow": None}
        full["depth"][r0 + rays] = cs["depth"]
        full["alpha"][r0 + rays] = cs["alpha"]
        per_scene.append((sc, cams, bi, rays, cs))
    tc = {k: torch.as_tensor(v, device=DEV).contiguous() for k, v in full.items()}
    tc["normal"] = tc["flow"] = None
    grads = b.backward(outs, tc, grads)
    torch.cuda.synchronize()
    for i, (sc, cams, bi, rays, cs) in enumerate(per_scene):
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        _, gref, _ = O.render_workload_view(sc, cams, bi, w.eta, rays=rays, cot=cs)
        gs = {"means": grads["means"][g0:g1], "prec": grads["prec"][g0:g1], "weights": grads["weights"][g0:g1],
              "betas": grads["betas"][i]}
        e = compare_grads(gs, gref)
        _say(f"[bench-config] scene {i} backward {fmt(e)}")
        assert_grads(e, f"bench configuration backward, scene {i}")


def test_colour_batch_vs_oracle(fmb, batch16):
    """The benchmark's colour leg through the tiled backward (variant 8, persistent): sigmoid colours
    on every scene of batch16, the forward colour of sampled rays, and one backward with depth,
    alpha and colour cotangents on sampled rays of every scene (zero elsewhere; depth and colour
    only where the oracle's alpha is at least 1e-3), against the oracle's gradient per scene."""
    w = batch16[0]
    b, _ = _batch_inputs(w, fmb)  # fresh parameters (other tests update the shared batch's)
    g = np.random.Generator(np.random.PCG64(94))
    qs = [(1.5 * g.standard_normal((s.n, 3))).astype(np.float32) for s in w.scenes]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    b.set_colors(t(np.concatenate(qs)))
    fmb.set_launch_config(batch=b, bwd_variant=8)
    outs = b.forward(b.alloc_outputs(normals=True, color=True))
    torch.cuda.synchronize()
    full = {"depth": np.zeros(b.n_rays, np.float32), "alpha": np.zeros(b.n_rays, np.float32),
            "color": np.zeros((b.n_rays, 3), np.float32)}
    per_scene = []
    for i, (sc, cams) in enumerate(zip(w.scenes, w.cameras)):
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        rays = np.sort(g.choice(r1 - r0, size=min(1000, r1 - r0), replace=False))
        ref, _, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays, colors=qs[i])
        sub = {k: (None if v is None else v[r0:r1]) for k, v in outs.items()}
        e = compare_forward(sub, ref, rays)
        e["color"] = normwise(to_np(outs["color"][r0:r1])[rays], ref["color"])
        _say(f"[colour-leg] scene {i} forward {fmt(e)}")
        assert_forward(e, f"colour leg scene {i}")
        assert e["color"] <= TOL_REL, (i, e["color"])
        hit = ref["alpha"] >= 1e-3
        cs = {"depth": (g.standard_normal(rays.size) * hit).astype(np.float32),
              "alpha": g.standard_normal(rays.size).astype(np.float32),
              "color": (g.standard_normal((rays.size, 3)) * hit[:, None]).astype(np.float32),
              "normal": None, "flow": None}
        for k in full:
            full[k][r0 + rays] = cs[k]
        per_scene.append((sc, cams, rays, cs))
    tc = {k: t(v) for k, v in full.items()}
    tc["normal"] = tc["flow"] = None
    grads = b.backward(outs, tc, b.alloc_grads(colors=True))
    torch.cuda.synchronize()
    assert fmb.launch_config(batch=b)["bwd_variant"] == 8
    for i, (sc, cams, rays, cs) in enumerate(per_scene):
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        _, gref, _ = O.render_workload_view(sc, cams, w.betas, w.eta, rays=rays, cot=cs, colors=qs[i])
        gs = {"means": grads["means"][g0:g1], "prec": grads["prec"][g0:g1], "weights": grads["weights"][g0:g1],
              "betas": grads["betas"][i]}
        e = compare_grads(gs, gref)
        e["colors"] = normwise(to_np(grads["colors"][g0:g1]), gref["colors"])
        _say(f"[colour-leg] scene {i} backward {fmt(e)}")
        assert_grads(e, f"colour leg backward, scene {i}")


def test_batch_with_a_large_scene(fmb):
    """A batch of a small scene and one of more than 256 Gaussians (which the kernel forms for large
    scenes take in pre-culled rounds): outputs and depth/alpha gradients of every scene equal
    per-scene launches bit for bit, and the large scene's match the oracle on sampled rays."""
    from tests.gpu_util import custom_scene
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    specs = [(40, [(64, 64), (48, 40)], 61, (0.05, 0.2)), (700, [(96, 128), (40, 72)], 62, (0.01, 0.05))]
    scenes = [custom_scene(n, views, seed=sd, s_range=sr) for n, views, sd, sr in specs]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    means = t(np.concatenate([sc.means for sc, _ in scenes]))
    prec = t(np.concatenate([sc.prec for sc, _ in scenes]))
    weights = t(np.concatenate([sc.weights for sc, _ in scenes]))
    tb = t(np.tile(betas, (2, 1)))
    cams = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, device=DEV) for _, c in scenes]
    b = fmb.Batch(means, prec, weights, tb, [1.0, 1.0], [sc.n for sc, _ in scenes], cams)
    _say(f"[large-batch] N={[sc.n for sc, _ in scenes]} P={b.n_rays}")
    outs = b.forward(b.alloc_outputs(normals=True))
    cot = _cotangents(b, 64, normals=False)
    grads = b.backward(outs, cot, b.alloc_grads())
    torch.cuda.synchronize()
    g = np.random.Generator(np.random.PCG64(65))
    for i, (sc, cm) in enumerate(scenes):
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        scene = fmb.Scene(means[g0:g1], prec[g0:g1], weights[g0:g1], tb[i], 1.0, cams[i])
        o = scene.render(normals=True)
        gi = scene.backward(o, cot["depth"][r0:r1], cot["alpha"][r0:r1], None)
        torch.cuda.synchronize()
        for k in ("depth", "alpha", "normal", "stash"):
            assert torch.equal(o[k], outs[k][r0:r1]), (i, k)
        for k in ("means", "prec", "weights"):
            assert torch.equal(gi[k], grads[k][g0:g1]), (i, k)
        assert torch.equal(gi["betas"], grads["betas"][i]), (i, "betas")
        if sc.n > 256:
            # (depth cotangents only on rays that see the scene, as in the other gradient tests)
            rays = np.sort(g.choice(r1 - r0, size=1500, replace=False))
            ref, _, _ = O.render_workload_view(sc, cm, betas, 1.0, rays=rays)
            cs = {"depth": to_np(cot["depth"][r0:r1])[rays] * (ref["alpha"] >= 1e-3),
                  "alpha": to_np(cot["alpha"][r0:r1])[rays], "normal": None, "flow": None}
            cs["depth"] = cs["depth"].astype(np.float32)
            _, gref, _ = O.render_workload_view(sc, cm, betas, 1.0, rays=rays, cot=cs)
            sub = {k: (None if v is None else v[r0:r1]) for k, v in outs.items()}
            e = compare_forward(sub, ref, rays)
            full = {k: np.zeros(r1 - r0, np.float32) for k in ("depth", "alpha")}
            for k in full:
                full[k][rays] = cs[k]
            gs = scene.backward(o, t(full["depth"]), t(full["alpha"]), None)
            torch.cuda.synchronize()
            eg = compare_grads(gs, gref)
            _say(f"[large-batch] scene {i} N={sc.n}: {fmt(e)} {fmt(eg)}")
            assert_forward(e, "large scene of a batch")
            assert_grads(eg, "large scene of a batch")


def test_graphs_dropped_when_stale(fmb):
    """Calls that change what the captured graphs launch (autotune, a pinned launch
    configuration, colours, a second flow target, a backward that rebuilds the work lists)
    drop them: the next replay reports FMB_ERR_STATE before launching anything, and a new
    capture replays like the eager calls again."""
    from tests.gpu_util import custom_scene
    scs = [custom_scene(n, views, seed=n, flow=True) for n, views in ((12, [(24, 20), (9, 31)]), (37, [(16, 16)]))]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()  # noqa: E731
    means = t(np.concatenate([s.means for s, _ in scs]))
    prec = t(np.concatenate([s.prec for s, _ in scs]))
    weights = t(np.concatenate([s.weights for s, _ in scs]))
    betas = t(np.tile(np.array([W.BETA1, W.BETA2], np.float32), (2, 1)))
    cams = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, c.w2c_b, c.intr_b, device=DEV) for _, c in scs]
    b = fmb.Batch(means, prec, weights, betas, [1.0, 1.0], [s.n for s, _ in scs], cams)
    outs = b.alloc_outputs(normals=True)
    grads = b.alloc_grads()
    cot = _cotangents(b, 47, normals=False)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()

    def capture_and_replay():
        b.capture(outs, cot, grads, st)
        with torch.cuda.stream(st):
            b.graph_launch(2, st)
        st.synchronize()

    def assert_stale(what):
        with pytest.raises(fmb.FmbError) as ei:
            b.graph_launch(2, st)
        assert ei.value.code == 6, what
        _say(f"[stale] after {what}: FMB_ERR_STATE")

    capture_and_replay()
    b.autotune(outs, cot, grads)
    torch.cuda.synchronize()
    assert_stale("autotune")
    capture_and_replay()
    fmb.set_launch_config(batch=b, bwd_variant=4)
    assert_stale("set_launch_config")
    capture_and_replay()
    q = t((np.random.Generator(np.random.PCG64(3)).standard_normal((means.shape[0], 3))).astype(np.float32))
    b.set_colors(q)
    assert_stale("set_colors")
    capture_and_replay()
    # an eager backward with a colour cotangent rebuilds the work lists with colour records
    outs_c = b.alloc_outputs(normals=True, color=True)
    grads_c = b.alloc_grads(colors=True)
    b.forward(outs_c)
    cot_c = dict(cot)
    cot_c["color"] = t(np.zeros((b.n_rays, 3), np.float32))
    b.backward(outs_c, cot_c, grads_c)
    torch.cuda.synchronize()
    assert_stale("a backward with a colour cotangent")
    b.set_colors(None)
    # a fresh capture replays like the eager calls
    capture_and_replay()
    ref_o = b.forward(b.alloc_outputs(normals=True))
    ref_g = b.backward(ref_o, cot, b.alloc_grads())
    torch.cuda.synchronize()
    for k in ("depth", "alpha", "normal"):
        assert torch.equal(outs[k], ref_o[k]), k
    for k in ("means", "prec", "weights", "betas"):
        assert torch.equal(grads[k], ref_g[k]), k
