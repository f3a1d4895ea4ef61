"""GPU split statistic (Sec. 8) against the oracle: lbar_i = (1/M) sum_j L_j w_ji over a random
minibatch of rays, for both blend models and for a batch of scenes."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import assert_forward, compare_forward, normwise, to_np

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


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()


def _minibatch(cams, frac, seed):
    """Explicit rays through random sub-pixel positions of every view: about `frac` of the pixels."""
    g = np.random.Generator(np.random.PCG64(seed))
    counts = np.maximum(1, (cams.hw[:, 0] * cams.hw[:, 1] * frac).astype(np.int64)).astype(np.int32)
    views = np.repeat(np.arange(cams.v), counts).astype(np.int32)
    p = int(counts.sum())
    hw = cams.hw[views].astype(np.float64)
    px = np.stack([g.uniform(0, 1, p) * hw[:, 1], g.uniform(0, 1, p) * hw[:, 0]], axis=1)
    k = cams.intr[views].astype(np.float64)
    dc = np.stack([(px[:, 0] - k[:, 2]) / k[:, 0], (px[:, 1] - k[:, 3]) / k[:, 1], np.ones(p)], axis=1)
    rot = cams.w2c[views, :, :3].astype(np.float64)
    dirs = np.einsum("pji,pj->pi", rot, dc).astype(np.float32)
    return counts, views, dirs


@pytest.mark.parametrize("model", ["blend", "composite"])
def test_split_statistic(fmb, model):
    w = W.make_config("fwdbwd128")
    sc, cams = w.scenes[0], w.cameras[0]
    counts, views, dirs = _minibatch(cams, 0.05, 70)
    p = int(counts.sum())
    _say(f"[split] fwdbwd128 {model}: {p} rays (5 %)")
    scene = fmb.Scene(_t(sc.means), _t(sc.prec), _t(sc.weights), _t(w.betas), w.eta)
    scene.set_rays(fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, device=DEV), counts, _t(dirs))
    scene.set_model(model)
    outs = scene.render(normals=False)
    o, v = O.dir_rays(views, dirs, cams.w2c)
    osc = O.OracleScene.of(sc.means, sc.prec, sc.weights, w.betas, w.eta)
    ref = O.render(osc, o, v, view=views, w2c_a=cams.w2c, intr_a=cams.intr, model=model)
    # the forward on these scattered explicit rays (a ray tile spans the whole view)
    ef = compare_forward(outs, ref, flow=False, normals=False)
    _say(f"[split] {model} forward: {ef}")
    assert_forward(ef, f"{model} forward on explicit rays")
    g = np.random.Generator(np.random.PCG64(71))
    # a per-ray loss that, like the reconstruction loss, vanishes where the ray sees nothing
    loss = (ref["alpha"] * g.uniform(0.5, 2.0, p)).astype(np.float32)
    lbar = scene.split_statistic(_t(loss), outs)
    torch.cuda.synchronize()
    lref = O.split_statistic(osc, o, v, loss, model)
    e = normwise(to_np(lbar), lref)
    total = float(to_np(lbar).sum())
    _say(f"[split] {model}: normwise {e:.3e} sum {total:.6f} mean loss {loss.mean():.6f}")
    assert e <= 1e-4
    assert abs(total - float(loss.astype(np.float64).mean())) <= 1e-4 * float(loss.mean())


def test_split_statistic_full_scene(fmb):
    """Every ray of the largest scene of the 16-scene batch (83 Gaussians, 1.57e6 rays): the
    finalize then sums thousands of items per Gaussian (strided over the threads of its block,
    then a fixed tree), against the oracle over the same rays."""
    w = W.make_config("batch16")
    sc, cams = w.scenes[0], w.cameras[0]
    scene = fmb.Scene(_t(sc.means), _t(sc.prec), _t(sc.weights), _t(w.betas), w.eta,
                      fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, device=DEV))
    outs = scene.render(normals=False)
    g = np.random.Generator(np.random.PCG64(73))
    loss_t = _t(g.uniform(0.5, 2.0, scene.n_rays).astype(np.float32)) * outs["alpha"]
    lbar = scene.split_statistic(loss_t, outs)
    torch.cuda.synchronize()
    loss = to_np(loss_t)
    _say(f"[split-full] N={sc.n} P={scene.n_rays}")
    from workloads import pixel_indices
    view, row, col = pixel_indices(cams)
    o, v = O.pixel_rays(view, row, col, cams.w2c, cams.intr)
    osc = O.OracleScene.of(sc.means, sc.prec, sc.weights, w.betas, w.eta)
    lref = O.split_statistic(osc, o, v, loss, "blend")
    e = normwise(to_np(lbar), lref)
    _say(f"[split-full] normwise {e:.3e}")
    assert e <= 1e-4
    assert abs(float(to_np(lbar).sum()) - float(loss.astype(np.float64).mean())) <= 1e-4 * float(loss.mean())


def test_split_statistic_batch(fmb):
    """Batched statistic equals each scene's own, bit for bit."""
    w = W.make_config("batch16")
    idx = [1, 8, 14]
    scenes = [w.scenes[i] for i in idx]
    cams = [w.cameras[i] for i in idx]
    means = _t(np.concatenate([s.means for s in scenes]))
    prec = _t(np.concatenate([s.prec for s in scenes]))
    weights = _t(np.concatenate([s.weights for s in scenes]))
    betas = _t(np.tile(w.betas, (len(scenes), 1)))
    tc = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, device=DEV) for c in cams]
    b = fmb.Batch(means, prec, weights, betas, [w.eta] * len(scenes), [s.n for s in scenes], tc)
    outs = b.forward(b.alloc_outputs(normals=False))
    g = np.random.Generator(np.random.PCG64(72))
    loss = _t(g.uniform(0, 1, b.n_rays).astype(np.float32)) * outs["alpha"]
    lbar = b.split_statistic(loss, outs)
    torch.cuda.synchronize()
    _say(f"[split-batch] scenes {idx} P={b.n_rays}")
    for i in range(len(scenes)):
        r0, r1 = b.ray_off[i], b.ray_off[i + 1]
        g0, g1 = b.gauss_off[i], b.gauss_off[i + 1]
        s = fmb.Scene(means[g0:g1], prec[g0:g1], weights[g0:g1], betas[i], w.eta, tc[i])
        so = s.render(normals=False)
        li = s.split_statistic(loss[r0:r1].contiguous(), so)
        torch.cuda.synchronize()
        assert torch.equal(li, lbar[g0:g1]), i
