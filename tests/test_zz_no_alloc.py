"""GPU test of fmb_backward_noalloc, the backward that allocates no device memory: through the C ABI
its gradients equal fmb_backward's bit for bit, on two calls in a row (the second on a smaller
input), and a scene whose work exceeds the fixed workspace is refused before any launch."""

from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import custom_scene, make_scene

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
    return None if a is None else torch.as_tensor(np.ascontiguousarray(a), device=DEV).contiguous()


# (label, Gaussians, views, cotangent of the normals): the first call takes the general adjoint
# (normal cotangent), the second, smaller one the offset form
CASES = [("n90_two_views", 90, [(96, 80), (40, 33)], True), ("n13_small", 13, [(17, 23)], False)]


def test_noalloc_backward_equals_backward(fmb):
    betas = np.array([W.BETA1, W.BETA2], np.float32)
    for label, n, views, with_normal in CASES:
        sc, cams = custom_scene(n, views, seed=n, flow=True)
        scene, _ = make_scene(fmb, torch, sc, cams, betas, 1.0, DEV)
        outs = scene.render(normals=True)
        cot = W.random_cotangents(cams.n_rays, 3 + n, flow=True)
        args = (outs, _t(cot["depth"]), _t(cot["alpha"]), _t(cot["normal"]) if with_normal else None,
                _t(cot["flow"]))
        ref = scene.backward(*args)
        torch.cuda.synchronize()
        _say(f"[noalloc] {label}: N={n} P={cams.n_rays} normal cotangent={with_normal}")
        got = scene.backward(*args, grads={k: torch.full_like(v, float("nan")) for k, v in ref.items()
                                           if v is not None}, noalloc=True)
        torch.cuda.synchronize()
        for k in ("means", "prec", "weights", "betas"):
            assert torch.equal(got[k], ref[k]), (label, k)
        _say(f"[noalloc] {label}: gradients equal fmb_backward's bit for bit")
    # a scene whose work plan needs more than the fixed workspace: refused on the host
    w = W.make_config("large1080")
    sc, cams = w.scenes[0], w.cameras[0]
    scene, _ = make_scene(fmb, torch, sc, cams, w.betas, w.eta, DEV)
    p = cams.n_rays
    outs = {"depth": torch.zeros(p, device=DEV), "stash": torch.zeros(p, 8, device=DEV)}
    with pytest.raises(fmb.FmbError) as ei:
        scene.backward(outs, torch.zeros(p, device=DEV), torch.zeros(p, device=DEV), noalloc=True)
    assert ei.value.code == 2 and "FMB_NOALLOC_SCRATCH_BYTES" in str(ei.value), str(ei.value)
    _say(f"[noalloc] large1080 refused: {ei.value}")
