"""PyTorch front-end of the gfx950 renderer: device memory, streams and autograd.

Every number is computed by the HIP kernels behind include/fmb.h; this module only
allocates output tensors, passes pointers and the current HIP stream, and wires the
backward kernel into torch.autograd.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib

STASH = 8  # floats of per-ray softmax state kept for the backward pass
# Blend weights of Eq. (3): the two-parameter model (Eq. 7) or alpha compositing (Eq. 9-10).
MODELS = {"blend": 0, "composite": 1}


def _model_id(model: str) -> int:
    if model not in MODELS:
        raise ValueError(f"model must be one of {sorted(MODELS)}")
    return MODELS[model]


def _vp(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f32(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float32, device=device)
    return t.contiguous()


def _check_dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class Cameras:
    """Views of one scene: w2c [V,3,4], intr [V,4] (fx, fy, cx, cy) on the GPU, hw [V,2]."""
    w2c: torch.Tensor
    intr: torch.Tensor
    hw: np.ndarray
    w2c_b: Optional[torch.Tensor] = None
    intr_b: Optional[torch.Tensor] = None
    w2c_c: Optional[torch.Tensor] = None   # optional second flow target (backward flow)
    intr_c: Optional[torch.Tensor] = None

    @classmethod
    def from_numpy(cls, w2c, intr, hw, w2c_b=None, intr_b=None, device="cuda", w2c_c=None,
                   intr_c=None) -> "Cameras":
        opt = lambda a: None if a is None else _dev_f32(a, device)  # noqa: E731
        return cls(_dev_f32(w2c, device), _dev_f32(intr, device),
                   np.ascontiguousarray(np.asarray(hw, dtype=np.int32)), opt(w2c_b), opt(intr_b),
                   opt(w2c_c), opt(intr_c))

    @property
    def flow_cols(self) -> int:
        return 0 if self.w2c_b is None else (4 if self.w2c_c is not None else 2)

    @property
    def v(self) -> int:
        return int(self.hw.shape[0])

    @property
    def n_rays(self) -> int:
        return int(np.sum(self.hw[:, 0].astype(np.int64) * self.hw[:, 1]))

    @property
    def has_flow(self) -> bool:
        return self.w2c_b is not None


class Scene:
    """A handle of the C ABI scene bound to (means, prec, weights, betas) and cameras."""

    def __init__(self, means, prec, weights, betas, eta: float = 1.0,
                 cameras: Optional[Cameras] = None):
        for t, nm in ((means, "means"), (prec, "prec"), (weights, "weights"), (betas, "betas")):
            _check_dev(t, nm)
        self.n = int(means.shape[0])
        if tuple(means.shape) != (self.n, 3) or tuple(prec.shape) != (self.n, 6) \
                or tuple(weights.shape) != (self.n,) or betas.numel() != 2:
            raise ValueError("expected means [N,3], prec [N,6], weights [N], betas [2]")
        self.device = means.device
        self.eta = float(eta)
        self._keep = (means, prec, weights, betas)
        h = ctypes.c_void_p()
        _lib.call("fmb_scene_create", ctypes.byref(h), self.n, _vp(means), _vp(prec), _vp(weights),
                  _vp(betas), ctypes.c_float(self.eta))
        self._h = h
        self.cameras = None
        self.model = "blend"
        if cameras is not None:
            self.set_cameras(cameras)

    @property
    def handle(self):
        return self._h

    def set_colors(self, colors: Optional[torch.Tensor]):
        """Per-Gaussian colours [N,3] (unconstrained; rendered as sigmoid), or None."""
        if colors is not None:
            _check_dev(colors, "colors")
            if tuple(colors.shape) != (self.n, 3):
                raise ValueError("colors must be [N,3]")
        _lib.call("fmb_set_colors", self._h, None, _vp(colors))
        self._colors = colors

    def set_model(self, model: str):
        """"blend" (two-parameter weights, Eq. 7) or "composite" (zero-parameter alpha
        compositing, Eq. 9-10; any number of Gaussians)."""
        _lib.call("fmb_set_model", self._h, None, _model_id(model))
        self.model = model

    def split_statistic(self, loss: torch.Tensor, outs: dict, lbar: Optional[torch.Tensor] = None):
        """lbar_i = (1/M) sum_j loss_j w_ji over this scene's M rays (Sec. 8); `outs` is the
        forward result (its stash) for the same parameters and model."""
        _check_dev(loss, "loss")
        out = lbar if lbar is not None else torch.empty(self.n, device=loss.device)
        _lib.call("fmb_split_statistic", self._h, None, _vp(loss), _vp(outs["stash"]), _vp(out),
                  _stream(loss.device))
        return out

    def rebind(self, means, prec, weights, betas):
        for t, nm in ((means, "means"), (prec, "prec"), (weights, "weights"), (betas, "betas")):
            _check_dev(t, nm)
        if means.shape[0] != self.n:
            raise ValueError("rebind needs the same number of Gaussians")
        _lib.call("fmb_scene_rebind", self._h, _vp(means), _vp(prec), _vp(weights), _vp(betas))
        self._keep = (means, prec, weights, betas)

    def set_cameras(self, cams: Cameras):
        hw = np.ascontiguousarray(cams.hw, dtype=np.int32)
        _lib.call("fmb_set_cameras", self._h, cams.v, _vp(cams.w2c), _vp(cams.intr),
                  hw.ctypes.data_as(ctypes.c_void_p), _vp(cams.w2c_b), _vp(cams.intr_b))
        if cams.w2c_c is not None:
            _lib.call("fmb_set_flow_pose2", self._h, None, _vp(cams.w2c_c), _vp(cams.intr_c))
        self.cameras = cams
        self._hw = hw

    def set_rays(self, cams: Cameras, counts, dirs: torch.Tensor):
        """Render an explicit ray minibatch: counts[k] rays of view k (view-major, contiguous),
        directions dirs [P,3] on the GPU (normalised by the kernels)."""
        _check_dev(dirs, "dirs")
        cnt = np.ascontiguousarray(np.asarray(counts, dtype=np.int32))
        if dirs.shape != (int(cnt.sum()), 3):
            raise ValueError("dirs must be [sum(counts), 3]")
        _lib.call("fmb_set_rays", self._h, int(cnt.shape[0]), _vp(cams.w2c), _vp(cams.intr),
                  cnt.ctypes.data_as(ctypes.c_void_p), _vp(dirs), _vp(cams.w2c_b), _vp(cams.intr_b))
        if cams.w2c_c is not None:
            _lib.call("fmb_set_flow_pose2", self._h, None, _vp(cams.w2c_c), _vp(cams.intr_c))
        self.cameras = cams
        self._dirs = dirs
        self._hw = cnt

    @property
    def n_rays(self) -> int:
        return int(_lib.load().fmb_num_rays(self._h))

    def render(self, normals: bool = True, flow: Optional[bool] = None, stash: bool = True,
               out: Optional[dict] = None, color: Optional[bool] = None) -> dict:
        if self.cameras is None:
            raise RuntimeError("set_cameras first")
        flow = self.cameras.has_flow if flow is None else flow
        color = (getattr(self, "_colors", None) is not None) if color is None else color
        p = self.n_rays
        o = out or {}
        dev = self.device
        depth = o.get("depth") if o.get("depth") is not None else torch.empty(p, device=dev)
        alpha = o.get("alpha") if o.get("alpha") is not None else torch.empty(p, device=dev)
        normal = None
        if normals:
            normal = o.get("normal") if o.get("normal") is not None else torch.empty(p, 3, device=dev)
        fl = None
        if flow:
            fl = o.get("flow") if o.get("flow") is not None else torch.empty(p, self.cameras.flow_cols,
                                                                             device=dev)
        col = None
        if color:
            col = o.get("color") if o.get("color") is not None else torch.empty(p, 3, device=dev)
        st = None
        if stash:
            st = o.get("stash") if o.get("stash") is not None else torch.empty(p, STASH, device=dev)
        _lib.call("fmb_render", self._h, _vp(depth), _vp(alpha), _vp(normal), _vp(fl), _vp(col), _vp(st),
                  _stream(dev))
        return {"depth": depth, "alpha": alpha, "normal": normal, "flow": fl, "color": col, "stash": st}

    @staticmethod
    def quality(outs: dict) -> torch.Tensor:
        """max_i of the normalised blend weights per ray (the Sec. 6 direct-intersection test
        max_i w_i > eps for point export), read from the stash."""
        return outs["stash"][:, 1]

    def backward(self, outs: dict, g_depth=None, g_alpha=None, g_normal=None, g_flow=None,
                 grads: Optional[dict] = None, g_color=None, noalloc: bool = False) -> dict:
        """Gradients of the cotangent-weighted outputs (fmb_backward; with `noalloc`,
        fmb_backward_noalloc: the same results from the library's fixed device workspace)."""
        dev = self.device
        g = grads or {}
        gm = g.get("means") if g.get("means") is not None else torch.empty(self.n, 3, device=dev)
        gp = g.get("prec") if g.get("prec") is not None else torch.empty(self.n, 6, device=dev)
        gw = g.get("weights") if g.get("weights") is not None else torch.empty(self.n, device=dev)
        gb = g.get("betas") if g.get("betas") is not None else torch.empty(2, device=dev)
        gc = None
        if g_color is not None:
            gc = g.get("colors") if g.get("colors") is not None else torch.empty(self.n, 3, device=dev)
        cot = [None if c is None else c.contiguous() for c in (g_depth, g_alpha, g_normal, g_flow, g_color)]
        _lib.call("fmb_backward_noalloc" if noalloc else "fmb_backward", self._h, *[_vp(c) for c in cot],
                  _vp(outs["depth"]),
                  _vp(outs.get("color")), _vp(outs["stash"]), _vp(gm), _vp(gp), _vp(gw), _vp(gc), _vp(gb),
                  _stream(dev))
        return {"means": gm, "prec": gp, "weights": gw, "betas": gb, "colors": gc}

    def validate(self) -> int:
        bad = ctypes.c_int32(0)
        _lib.call("fmb_validate", self._h, ctypes.byref(bad), _stream(self.device))
        return int(bad.value)

    def autotune(self, outs: dict, cot: dict, grads: dict, cache_path: Optional[str] = None):
        """Pick the fastest compiled tile variants for these outputs and cotangents."""
        _lib.call("fmb_autotune", self._h, None, *_tune_args(outs, cot, grads),
                  None if cache_path is None else cache_path.encode(), _stream(self.device))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
                _lib.load().fmb_scene_destroy(h)
            except Exception:
                pass
            self._h = None


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene: Scene, normals: bool, means, prec, weights, betas, colors):
        scene.rebind(means.detach().contiguous(), prec.detach().contiguous(),
                     weights.detach().contiguous(), betas.detach().contiguous())
        scene.set_colors(None if colors is None else colors.detach().contiguous())
        outs = scene.render(normals=normals, color=colors is not None)
        ctx.scene = scene
        ctx.outs = outs
        ctx.has_colors = colors is not None
        ctx.save_for_backward(means, prec, weights, betas, colors)
        empty = outs["depth"].new_zeros(0)
        nr = outs["normal"] if outs["normal"] is not None else empty
        fl = outs["flow"] if outs["flow"] is not None else empty
        co = outs["color"] if outs["color"] is not None else empty
        ctx.mark_non_differentiable(outs["stash"])
        # an output the loss does not use passes no cotangent (not zeros), so that, e.g., a
        # loss without the normals takes the backward without the normal adjoint
        ctx.set_materialize_grads(False)
        return outs["depth"], outs["alpha"], nr, fl, co

    @staticmethod
    def backward(ctx, g_depth, g_alpha, g_normal, g_flow, g_color):
        scene = ctx.scene
        outs = ctx.outs
        means, prec, weights, betas, colors = ctx.saved_tensors
        scene.rebind(means.detach().contiguous(), prec.detach().contiguous(),
                     weights.detach().contiguous(), betas.detach().contiguous())
        scene.set_colors(None if colors is None else colors.detach().contiguous())
        use = lambda g, o: g if (o is not None and g is not None and g.numel() > 0) else None  # noqa: E731
        gr = scene.backward(outs, use(g_depth, outs["depth"]), use(g_alpha, outs["alpha"]),
                            use(g_normal, outs["normal"]), use(g_flow, outs["flow"]),
                            g_color=use(g_color, outs["color"]))
        gcol = gr["colors"] if ctx.has_colors else None
        if ctx.has_colors and gcol is None:
            gcol = torch.zeros_like(colors)
        return None, None, gr["means"], gr["prec"], gr["weights"], gr["betas"], gcol


def render(scene: Scene, means, prec, weights, betas, normals: bool = True, colors=None):
    """Differentiable render: returns (depth [P], alpha [P], normal [P,3] or empty, flow [P,2] or
    empty, colour [P,3] or empty); gradients flow to means, prec, weights, betas and colours
    through the HIP adjoint kernel."""
    return _RenderFn.apply(scene, normals, means, prec, weights, betas, colors)


def _tune_args(outs, cot, grads):
    return (_vp(outs["depth"]), _vp(outs["alpha"]), _vp(outs.get("normal")), _vp(outs.get("flow")),
            _vp(outs.get("color")), _vp(outs["stash"]), _vp(cot.get("depth")), _vp(cot.get("alpha")),
            _vp(cot.get("normal")), _vp(cot.get("flow")), _vp(cot.get("color")), _vp(grads["means"]),
            _vp(grads["prec"]), _vp(grads["weights"]), _vp(grads.get("colors")), _vp(grads["betas"]))


class Batch:
    """Many scenes rendered by the persistent batched kernels (one launch per pass)."""

    def __init__(self, means, prec, weights, betas, eta: Sequence[float], n_per_scene: Sequence[int],
                 cams: List[Cameras]):
        for t, nm in ((means, "means"), (prec, "prec"), (weights, "weights"), (betas, "betas")):
            _check_dev(t, nm)
        self.s = len(n_per_scene)
        self.device = means.device
        self.n_host = np.ascontiguousarray(np.asarray(n_per_scene, dtype=np.int32))
        self.v_host = np.ascontiguousarray(np.asarray([c.v for c in cams], dtype=np.int32))
        self.eta = np.ascontiguousarray(np.asarray(eta, dtype=np.float32))
        self.w2c = torch.cat([c.w2c.reshape(-1, 12) for c in cams]).contiguous()
        self.intr = torch.cat([c.intr.reshape(-1, 4) for c in cams]).contiguous()
        self.hw = np.ascontiguousarray(np.concatenate([c.hw for c in cams]).astype(np.int32))
        flows = [c.has_flow for c in cams]
        if any(flows) and not all(flows):
            raise ValueError("either every scene or none has a second pose")
        self.w2c_b = torch.cat([c.w2c_b.reshape(-1, 12) for c in cams]).contiguous() if all(flows) else None
        self.intr_b = torch.cat([c.intr_b.reshape(-1, 4) for c in cams]).contiguous() if all(flows) else None
        second = [c.w2c_c is not None for c in cams]
        if any(second) and not all(second):
            raise ValueError("either every scene or none has a second flow target")
        self.w2c_c = torch.cat([c.w2c_c.reshape(-1, 12) for c in cams]).contiguous() if all(second) else None
        self.intr_c = torch.cat([c.intr_c.reshape(-1, 4) for c in cams]).contiguous() if all(second) else None
        self.n_total = int(self.n_host.sum())
        self.model = "blend"
        self._keep = (means, prec, weights, betas)
        h = ctypes.c_void_p()
        _lib.call("fmb_batch_create", ctypes.byref(h), self.s, self.n_host.ctypes.data_as(ctypes.c_void_p),
                  self.v_host.ctypes.data_as(ctypes.c_void_p), _vp(means), _vp(prec), _vp(weights),
                  _vp(betas), self.eta.ctypes.data_as(ctypes.c_void_p), _vp(self.w2c), _vp(self.intr),
                  self.hw.ctypes.data_as(ctypes.c_void_p), _vp(self.w2c_b), _vp(self.intr_b))
        self._h = h
        if self.w2c_c is not None:
            _lib.call("fmb_set_flow_pose2", None, h, _vp(self.w2c_c), _vp(self.intr_c))
        lib = _lib.load()
        self.n_rays = int(lib.fmb_batch_num_rays(h))
        self.ray_off = [int(lib.fmb_batch_ray_offset(h, i)) for i in range(self.s + 1)]
        self.gauss_off = [int(lib.fmb_batch_gauss_offset(h, i)) for i in range(self.s + 1)]

    @property
    def has_flow(self) -> bool:
        return self.w2c_b is not None

    @property
    def flow_cols(self) -> int:
        return 0 if self.w2c_b is None else (4 if self.w2c_c is not None else 2)

    def set_colors(self, colors: Optional[torch.Tensor]):
        """Per-Gaussian colours [sum N, 3] (unconstrained), or None."""
        if colors is not None:
            _check_dev(colors, "colors")
        _lib.call("fmb_set_colors", None, self._h, _vp(colors))
        self._colors = colors

    def set_model(self, model: str):
        """"blend" or "composite" for every scene of the batch (see Scene.set_model)."""
        _lib.call("fmb_set_model", None, self._h, _model_id(model))
        self.model = model

    def split_statistic(self, loss: torch.Tensor, outs: dict, lbar: Optional[torch.Tensor] = None):
        """Scene.split_statistic for every scene of the batch: lbar [sum N]."""
        _check_dev(loss, "loss")
        out = lbar if lbar is not None else torch.empty(self.n_total, device=loss.device)
        _lib.call("fmb_split_statistic", None, self._h, _vp(loss), _vp(outs["stash"]), _vp(out),
                  _stream(loss.device))
        return out

    def alloc_outputs(self, normals=True, color=False):
        p, dev = self.n_rays, self.device
        return {"depth": torch.empty(p, device=dev), "alpha": torch.empty(p, device=dev),
                "normal": torch.empty(p, 3, device=dev) if normals else None,
                "flow": torch.empty(p, self.flow_cols, device=dev) if self.has_flow else None,
                "color": torch.empty(p, 3, device=dev) if color else None,
                "stash": torch.empty(p, STASH, device=dev)}

    def alloc_grads(self, colors=False):
        n, dev = self.n_total, self.device
        return {"means": torch.empty(n, 3, device=dev), "prec": torch.empty(n, 6, device=dev),
                "weights": torch.empty(n, device=dev), "betas": torch.empty(self.s, 2, device=dev),
                "colors": torch.empty(n, 3, device=dev) if colors else None}

    def forward(self, outs: dict):
        _lib.call("fmb_batch_forward", self._h, _vp(outs["depth"]), _vp(outs["alpha"]),
                  _vp(outs["normal"]), _vp(outs["flow"]), _vp(outs.get("color")), _vp(outs["stash"]),
                  _stream(self.device))
        return outs

    def forward_loss(self, outs: dict, depth_t, alpha_t, cot: dict, w_depth: float = 1.0):
        """forward() with the depth and alpha cotangents of the reconstruction loss (what
        loss_grad writes for them) computed in the same pass, into cot["depth"], cot["alpha"]."""
        _lib.call("fmb_batch_forward_loss", self._h, _vp(outs["depth"]), _vp(outs["alpha"]),
                  _vp(outs["normal"]), _vp(outs["flow"]), _vp(outs.get("color")), _vp(outs["stash"]),
                  _vp(depth_t.contiguous()), _vp(alpha_t.contiguous()), ctypes.c_float(w_depth),
                  _vp(cot["depth"]), _vp(cot["alpha"]), _stream(self.device))
        return outs

    def backward(self, outs: dict, cot: dict, grads: dict):
        _lib.call("fmb_batch_backward", self._h, _vp(cot.get("depth")), _vp(cot.get("alpha")),
                  _vp(cot.get("normal")), _vp(cot.get("flow")), _vp(cot.get("color")), _vp(outs["depth"]),
                  _vp(outs.get("color")), _vp(outs["stash"]), _vp(grads["means"]), _vp(grads["prec"]),
                  _vp(grads["weights"]), _vp(grads.get("colors")), _vp(grads["betas"]), _stream(self.device))
        return grads

    def capture(self, outs: dict, cot: dict, grads: dict, stream: torch.cuda.Stream):
        _lib.call("fmb_batch_capture", self._h, _vp(outs["depth"]), _vp(outs["alpha"]),
                  _vp(outs["normal"]), _vp(outs["flow"]), _vp(outs.get("color")), _vp(outs["stash"]),
                  _vp(cot.get("depth")), _vp(cot.get("alpha")), _vp(cot.get("normal")), _vp(cot.get("flow")),
                  _vp(cot.get("color")), _vp(grads["means"]), _vp(grads["prec"]), _vp(grads["weights"]),
                  _vp(grads.get("colors")), _vp(grads["betas"]), ctypes.c_void_p(stream.cuda_stream))

    def graph_launch(self, which: int = 2, stream: Optional[torch.cuda.Stream] = None):
        """Replay the captured forward (0), backward (1) or both (2)."""
        st = stream.cuda_stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _lib.call("fmb_batch_graph_launch", self._h, int(which), ctypes.c_void_p(st))

    def autotune(self, outs: dict, cot: dict, grads: dict, cache_path: Optional[str] = None):
        """Pick the fastest compiled tile variants for these outputs and cotangents."""
        _lib.call("fmb_autotune", None, self._h, *_tune_args(outs, cot, grads),
                  None if cache_path is None else cache_path.encode(), _stream(self.device))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
                _lib.load().fmb_batch_destroy(h)
            except Exception:
                pass
            self._h = None


def set_launch_config(scene: Optional["Scene"] = None, batch: Optional["Batch"] = None, fwd_variant: int = 3,
                      bwd_variant: int = 8, fwd_grid_mult: int = 1, bwd_grid_mult: int = 1):
    """Pin the tile variants and persistent-grid multipliers (see launch_config)."""
    _lib.call("fmb_set_config", scene.handle if scene is not None else None,
              batch._h if batch is not None else None, int(fwd_variant), int(bwd_variant), int(fwd_grid_mult),
              int(bwd_grid_mult))


def launch_config(scene: Optional["Scene"] = None, batch: Optional["Batch"] = None) -> dict:
    """Tile variants, persistent-grid multipliers and work-item counts in use."""
    out = (ctypes.c_int32 * 8)()
    _lib.call("fmb_get_config", scene.handle if scene is not None else None,
              batch._h if batch is not None else None, out)
    keys = ("fwd_variant", "fwd_rays_per_item", "bwd_variant", "bwd_rays_per_tile", "fwd_grid_mult",
            "bwd_grid_mult", "fwd_items", "bwd_items")
    return dict(zip(keys, list(out)))


def loss_grad(outs: dict, depth_t, alpha_t, flow_t=None, w_depth: float = 1.0, w_flow: float = 1.0,
              flow_norm: int = 2, cot: Optional[dict] = None, block_loss: Optional[torch.Tensor] = None,
              color_t=None, w_color: float = 1.0) -> dict:
    """Cotangents of the mask-weighted reconstruction loss (BCE alpha + w_depth alpha* L1 depth
    + w_color alpha* L1 colour + w_flow alpha* flow term, averaged over rays) in one HIP kernel."""
    p = int(outs["depth"].numel())
    dev = outs["depth"].device
    c = cot if cot is not None else {}
    gd = c.get("depth") if c.get("depth") is not None else torch.empty(p, device=dev)
    ga = c.get("alpha") if c.get("alpha") is not None else torch.empty(p, device=dev)
    gf = gc = None
    if flow_t is not None:
        gf = c.get("flow") if c.get("flow") is not None else torch.empty_like(outs["flow"])
    if color_t is not None:
        gc = c.get("color") if c.get("color") is not None else torch.empty(p, 3, device=dev)
    _lib.call("fmb_loss_grad", p, _vp(outs["depth"]), _vp(outs["alpha"]),
              _vp(outs["flow"] if flow_t is not None else None),
              _vp(outs["color"] if color_t is not None else None), _vp(depth_t), _vp(alpha_t), _vp(flow_t),
              _vp(color_t), ctypes.c_float(w_depth), ctypes.c_float(w_flow), int(flow_norm),
              int(outs["flow"].shape[1]) if flow_t is not None else 2,
              ctypes.c_float(w_color), _vp(gd), _vp(ga), _vp(gf), _vp(gc), _vp(block_loss), _stream(dev))
    return {"depth": gd, "alpha": ga, "normal": None, "flow": gf, "color": gc}


def timing_enable(on: bool = True):
    _lib.call("fmb_timing_enable", 1 if on else 0)


def kernel_times(reset: bool = False) -> dict:
    buf = (ctypes.c_double * 6)()
    _lib.call("fmb_kernel_times", buf, 1 if reset else 0)
    return {"fwd_ms": buf[0], "bwd_ms": buf[1], "fin_ms": buf[2],
            "n_fwd": int(buf[3]), "n_bwd": int(buf[4]), "n_fin": int(buf[5])}
