"""ctypes front-end of the FP64 oracle (fmb_oracle.c).

TEST INFRASTRUCTURE: used by the tests, the smoke check and the CPU-baseline leg
of the benchmark only.  Inputs are the float32 values the GPU path consumes,
upcast to float64; all arithmetic is double precision.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmb_oracle.c")
_LIB = os.path.join(_HERE, "libfmb_oracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def _configure(lib):
    lib.fmbo_version.restype = ctypes.c_int
    lib.fmbo_pixel_rays.argtypes = [ctypes.c_int64, _I, _I, _I, _D, _D, _D, _D]
    lib.fmbo_dir_rays.argtypes = [ctypes.c_int64, _I, _D, _D, _D, _D]
    lib.fmbo_project.argtypes = [ctypes.c_int64, _I, _D, _D, _D, _D]
    common = [ctypes.c_int32, _D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int64, _D, _D, _I,
              _D, _D, _D, _D]
    lib.fmbo_render.argtypes = common + [_D, _D, _D, _D, _D, ctypes.c_int]
    lib.fmbo_render.restype = ctypes.c_int
    lib.fmbo_backward.argtypes = common + [_D, _D, _D, _D, _D, _D, _D, _D, _D, _D, ctypes.c_int]
    lib.fmbo_backward.restype = ctypes.c_int
    lib.fmbo_render_model.argtypes = [ctypes.c_int32] + lib.fmbo_render.argtypes
    lib.fmbo_render_model.restype = ctypes.c_int
    lib.fmbo_backward_model.argtypes = [ctypes.c_int32] + lib.fmbo_backward.argtypes
    lib.fmbo_backward_model.restype = ctypes.c_int
    lib.fmbo_ray_weights.argtypes = [ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _D, ctypes.c_double,
                                     _D, _D, _D]
    lib.fmbo_ray_weights.restype = ctypes.c_int
    lib.fmbo_split_statistic.argtypes = [ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _D, ctypes.c_double,
                                         ctypes.c_int64, _D, _D, _D, _D, ctypes.c_int]
    lib.fmbo_split_statistic.restype = ctypes.c_int
    lib.fmbo_ray_terms.argtypes = [ctypes.c_int32, _D, _D, _D, _D, ctypes.c_double, _D, _D,
                                   _D, _D, _D, _D]
    return lib


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def use_library(path):
    """Route every oracle call through another build of fmb_oracle.c (a planted-mistake
    copy in the mutation tests); returns the previous handle for `restore_library`."""
    global _lib
    prev = load()
    _lib = _configure(ctypes.CDLL(path))
    return prev


def restore_library(prev):
    global _lib
    _lib = prev


def _d(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, typ=_D):
    return None if a is None else a.ctypes.data_as(typ)


def _i32(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


@dataclass
class OracleScene:
    """Gaussians (float64 copies), optional unconstrained colours [N,3], blend parameters."""
    means: np.ndarray
    prec: np.ndarray
    weights: np.ndarray
    betas: np.ndarray
    eta: float = 1.0
    colors: Optional[np.ndarray] = None

    @classmethod
    def of(cls, means, prec, weights, betas, eta=1.0, colors=None) -> "OracleScene":
        return cls(_d(means).reshape(-1, 3), _d(prec).reshape(-1, 6), _d(weights).reshape(-1),
                   _d(betas).reshape(2), float(eta),
                   None if colors is None else _d(colors).reshape(-1, 3))

    @property
    def n(self) -> int:
        return self.means.shape[0]


def pixel_rays(view, row, col, w2c, intr):
    """Ray origins and unit directions [P,3] through pixel centres (float64)."""
    lib = load()
    view, row, col = _i32(view), _i32(row), _i32(col)
    w2c, intr = _d(w2c).reshape(-1, 12), _d(intr).reshape(-1, 4)
    p = view.shape[0]
    o = np.empty((p, 3))
    v = np.empty((p, 3))
    lib.fmbo_pixel_rays(p, _p(view, _I), _p(row, _I), _p(col, _I), _p(w2c), _p(intr), _p(o), _p(v))
    return o, v


def dir_rays(view, dirs, w2c):
    lib = load()
    view = _i32(view)
    dirs, w2c = _d(dirs).reshape(-1, 3), _d(w2c).reshape(-1, 12)
    p = view.shape[0]
    o = np.empty((p, 3))
    v = np.empty((p, 3))
    lib.fmbo_dir_rays(p, _p(view, _I), _p(dirs), _p(w2c), _p(o), _p(v))
    return o, v


def project(view, pts, w2c, intr):
    lib = load()
    view = _i32(view)
    pts, w2c, intr = _d(pts).reshape(-1, 3), _d(w2c).reshape(-1, 12), _d(intr).reshape(-1, 4)
    uv = np.empty((view.shape[0], 2))
    lib.fmbo_project(view.shape[0], _p(view, _I), _p(pts), _p(w2c), _p(intr), _p(uv))
    return uv


def _cams(view, w2c_a, intr_a, w2c_b, intr_b):
    view = _i32(view)
    a = _d(w2c_a).reshape(-1, 12) if w2c_a is not None else None
    ia = _d(intr_a).reshape(-1, 4) if intr_a is not None else None
    b = _d(w2c_b).reshape(-1, 12) if w2c_b is not None else None
    ib = _d(intr_b).reshape(-1, 4) if intr_b is not None else None
    return view, a, ia, b, ib


MODELS = {"blend": 0, "composite": 1}


def _model(model):
    if model not in MODELS:
        raise ValueError(f"model must be one of {sorted(MODELS)}")
    return MODELS[model]


def render(scene: OracleScene, orig, dirs, view=None, w2c_a=None, intr_a=None, w2c_b=None,
           intr_b=None, n_threads: int = 0, w2c_c=None, intr_c=None, model: str = "blend"):
    """Forward pass over explicit rays; returns dict(depth, alpha, normal, flow, color).

    model "blend": the two-parameter weights of Eq. (7); "composite": the zero-parameter
    alpha-compositing weights of Eq. (9)-(10) (betas and eta unused).

    With a third pose (w2c_c, intr_c) the flow has 4 columns per ray: the flow to pose B and
    the flow to pose C (Sec. 5 estimates forward and backward flow for every ray); each is the
    same definition, pi_X(p) - pi_A(p), evaluated for its own target pose."""
    if w2c_c is not None:
        if w2c_b is None:
            raise ValueError("a third pose needs the second one")
        out = render(scene, orig, dirs, view, w2c_a, intr_a, w2c_b, intr_b, n_threads, model=model)
        back = render(scene, orig, dirs, view, w2c_a, intr_a, w2c_c, intr_c, n_threads, model=model)
        out["flow"] = np.concatenate([out["flow"], back["flow"]], axis=1)
        return out
    lib = load()
    orig, dirs = _d(orig).reshape(-1, 3), _d(dirs).reshape(-1, 3)
    p = orig.shape[0]
    view, a, ia, b, ib = _cams(view, w2c_a, intr_a, w2c_b, intr_b)
    out = {"depth": np.empty(p), "alpha": np.empty(p), "normal": np.empty((p, 3)),
           "flow": np.empty((p, 2)) if b is not None else None,
           "color": np.empty((p, 3)) if scene.colors is not None else None}
    rc = lib.fmbo_render_model(_model(model), scene.n, _p(scene.means), _p(scene.prec), _p(scene.weights),
                         _p(scene.colors), _p(scene.betas), scene.eta, p, _p(orig), _p(dirs),
                         _p(view, _I), _p(a), _p(ia), _p(b), _p(ib), _p(out["depth"]),
                         _p(out["alpha"]), _p(out["normal"]), _p(out["flow"]), _p(out["color"]),
                         int(n_threads))
    if rc != 0:
        raise ValueError("oracle render rejected its arguments")
    return out


def backward(scene: OracleScene, orig, dirs, cot: dict, view=None, w2c_a=None, intr_a=None,
             w2c_b=None, intr_b=None, n_threads: int = 0, w2c_c=None, intr_c=None,
             model: str = "blend"):
    """Gradients of sum(cot . outputs) w.r.t. means [N,3], prec [N,6], weights [N], betas [2]
    (and colours [N,3] when the scene has them).

    With a third pose the flow cotangent has 4 columns; the objective is then the sum of the
    usual one (flow to B) and the flow-to-C term alone, so its gradient is the sum of the two
    gradients (linearity of the derivative)."""
    if w2c_c is not None:
        gf = np.asarray(cot["flow"], np.float64).reshape(-1, 4)
        first = dict(cot, flow=gf[:, :2])
        g1 = backward(scene, orig, dirs, first, view, w2c_a, intr_a, w2c_b, intr_b, n_threads,
                      model=model)
        g2 = backward(scene, orig, dirs, {"flow": gf[:, 2:]}, view, w2c_a, intr_a, w2c_c, intr_c,
                      n_threads, model=model)
        return {k: None if g1[k] is None else g1[k] + g2[k] for k in g1}
    lib = load()
    orig, dirs = _d(orig).reshape(-1, 3), _d(dirs).reshape(-1, 3)
    p = orig.shape[0]
    view, a, ia, b, ib = _cams(view, w2c_a, intr_a, w2c_b, intr_b)
    gd, ga = _d(cot.get("depth")), _d(cot.get("alpha"))
    gn, gf, gc = _d(cot.get("normal")), _d(cot.get("flow")), _d(cot.get("color"))
    n = scene.n
    out = {"means": np.empty((n, 3)), "prec": np.empty((n, 6)), "weights": np.empty(n),
           "betas": np.empty(2), "colors": np.empty((n, 3)) if scene.colors is not None else None}
    rc = lib.fmbo_backward_model(_model(model), n, _p(scene.means), _p(scene.prec), _p(scene.weights),
                           _p(scene.colors), _p(scene.betas), scene.eta, p, _p(orig), _p(dirs),
                           _p(view, _I), _p(a), _p(ia), _p(b), _p(ib), _p(gd), _p(ga), _p(gn),
                           _p(gf), _p(gc), _p(out["means"]), _p(out["prec"]), _p(out["weights"]),
                           _p(out["colors"]), _p(out["betas"]), int(n_threads))
    if rc != 0:
        raise ValueError("oracle backward rejected its arguments")
    return out


def blend_weights(scene: OracleScene, o, v, model: str = "blend"):
    """Normalised blend weights w_i / sum_j w_j of Eq. (3) along one ray."""
    lib = load()
    o, v = _d(o).reshape(3), _d(v).reshape(3)
    wt = np.empty(scene.n)
    rc = lib.fmbo_ray_weights(_model(model), scene.n, _p(scene.means), _p(scene.prec),
                              _p(scene.weights), _p(scene.betas), scene.eta, _p(o), _p(v), _p(wt))
    if rc != 0:
        raise ValueError("oracle ray_weights rejected its arguments")
    return wt


def max_weight(scene: OracleScene, orig, dirs, model: str = "blend"):
    """max_i of the normalised blend weights per ray: the direct-intersection quality of
    Sec. 6 (points with max_i w_i <= eps are rejected for mesh export).  Small inputs only:
    one call per ray."""
    orig, dirs = _d(orig).reshape(-1, 3), _d(dirs).reshape(-1, 3)
    return np.array([blend_weights(scene, orig[r], dirs[r], model).max() for r in range(orig.shape[0])])


def split_statistic(scene: OracleScene, orig, dirs, loss, model: str = "blend", n_threads: int = 0):
    """Average loss assigned to each Gaussian over a batch of M rays (Sec. 8):
    lbar_i = (1/M) sum_j L_j w_ji with w_ji the normalised blend weights of ray j."""
    lib = load()
    orig, dirs = _d(orig).reshape(-1, 3), _d(dirs).reshape(-1, 3)
    loss = _d(loss).reshape(-1)
    out = np.empty(scene.n)
    rc = lib.fmbo_split_statistic(_model(model), scene.n, _p(scene.means), _p(scene.prec), _p(scene.weights),
                                  _p(scene.betas), scene.eta, orig.shape[0], _p(orig), _p(dirs), _p(loss),
                                  _p(out), int(n_threads))
    if rc != 0:
        raise ValueError("oracle split_statistic rejected its arguments")
    return out


def prune_mask(weights, z=2.0):
    """Removal test of Sec. 8: lambda_i <= mean(lambda) - z std(lambda) (population std)."""
    w = np.asarray(weights, np.float64)
    return w <= w.mean() - z * w.std()


def split_mask(lbar, z=1.0):
    """Split test of Sec. 8: lbar_i >= mean(lbar) + z std(lbar)."""
    x = np.asarray(lbar, np.float64)
    return x >= x.mean() + z * x.std()


def split_gaussians(means, prec, weights, colors=None, noise_w=None, noise_c=None):
    """Split of Sec. 8 by the half-normal distribution: each Gaussian gives two with means
    mu +- sigma_1 sqrt(2/pi) v_1 (v_1 the dominant eigenvector of Sigma, sigma_1^2 its
    eigenvalue: sigma_1 is read as the standard deviation along v_1, the reading under which
    the shift is a length) and the same covariance with sigma_1 scaled by sqrt(1 - 2/pi);
    log-weights and unconstrained colours get the caller's noise.  v_1's largest-magnitude
    component is taken positive; child 2i is the + shift.  Returns float64 arrays."""
    means = np.asarray(means, np.float64)
    prec = np.asarray(prec, np.float64)
    n = means.shape[0]
    noise_w = np.zeros(2 * n) if noise_w is None else np.asarray(noise_w, np.float64)
    out = {"means": np.empty((2 * n, 3)), "prec": np.empty((2 * n, 6)), "weights": np.empty(2 * n),
           "colors": None if colors is None else np.empty((2 * n, 3))}
    for i in range(n):
        u = prec[i]
        U = np.array([[u[0], u[1], u[2]], [0.0, u[3], u[4]], [0.0, 0.0, u[5]]])
        cov = np.linalg.inv(U.T @ U)
        vals, vecs = np.linalg.eigh(cov)            # ascending
        v1 = vecs[:, -1]
        if v1[np.argmax(np.abs(v1))] < 0:
            v1 = -v1
        sigma1 = math.sqrt(vals[-1])
        vals2 = vals.copy()
        vals2[-1] = vals[-1] * (1.0 - 2.0 / math.pi)
        cov2 = vecs @ np.diag(vals2) @ vecs.T
        L = np.linalg.cholesky(np.linalg.inv(cov2))  # Sigma'^-1 = L L^T, U' = L^T
        Up = L.T
        for child, sgn in ((0, 1.0), (1, -1.0)):
            o = 2 * i + child
            out["means"][o] = means[i] + sgn * sigma1 * math.sqrt(2.0 / math.pi) * v1
            out["prec"][o] = [Up[0, 0], Up[0, 1], Up[0, 2], Up[1, 1], Up[1, 2], Up[2, 2]]
            out["weights"][o] = float(weights[i]) * math.exp(noise_w[o])
            if colors is not None:
                out["colors"][o] = np.asarray(colors[i], np.float64) + np.asarray(noise_c[o], np.float64)
    return out


def ray_terms(scene: OracleScene, o, v):
    """Per-Gaussian (t_i, d_i, z_i, n_i) of one ray."""
    lib = load()
    o, v = _d(o).reshape(3), _d(v).reshape(3)
    n = scene.n
    t, d, z, nrm = np.empty(n), np.empty(n), np.empty(n), np.empty((n, 3))
    lib.fmbo_ray_terms(n, _p(scene.means), _p(scene.prec), _p(scene.weights), _p(scene.betas),
                       scene.eta, _p(o), _p(v), _p(t), _p(d), _p(z), _p(nrm))
    return t, d, z, nrm


def render_workload_view(scene, cams, betas, eta, rays=None, n_threads: int = 0, cot=None,
                         colors=None, model: str = "blend"):
    """Render (and optionally differentiate) pixel rays of a workload camera set.

    `scene` has means/prec/weights (float32 arrays), `cams` has w2c, intr, hw and the
    optional second pose.  `rays` selects global ray indices (default: all).
    Returns (outputs, grads or None, (view, row, col)).
    """
    from workloads import pixel_indices  # input bookkeeping only
    view, row, col = pixel_indices(cams, rays)
    o, v = pixel_rays(view, row, col, cams.w2c, cams.intr)
    sc = OracleScene.of(scene.means, scene.prec, scene.weights, betas, eta, colors)
    kw = dict(view=view, w2c_a=cams.w2c, intr_a=cams.intr, w2c_b=cams.w2c_b, intr_b=cams.intr_b,
              n_threads=n_threads, w2c_c=getattr(cams, "w2c_c", None),
              intr_c=getattr(cams, "intr_c", None), model=model)
    out = render(sc, o, v, **kw)
    grads = backward(sc, o, v, cot, **kw) if cot is not None else None
    return out, grads, (view, row, col)


def loss_grad(depth, alpha, depth_t, alpha_t, flow=None, flow_t=None, w_depth=1.0, w_flow=1.0,
              flow_norm=2, color=None, color_t=None, w_color=1.0):
    """Reconstruction loss of Sec. 4 (Eq. 11-14) averaged over rays, and its gradient with respect
    to the rendered depth, alpha and flow (float64, straight from the definition):
      L = mean_r [ -(a* log a + (1 - a*) log(1 - a)),  a = clamp(alpha, 1e-6, 1 - 1e-6)   (Eq. 11)
                   + w_depth a* |depth - depth*|                        (mask-weighted L1)
                   + w_color a* |color - color*|_1                      (Eq. 12)
                   + w_flow a* |flow - flow*|_1 or squared L2 ]          (Eq. 13)
    The clamp passes the gradient where 1e-6 <= alpha <= 1 - 1e-6 (bounds as float32 values);
    d|x|/dx = sign(x)."""
    d, a = np.asarray(depth, np.float64), np.asarray(alpha, np.float64)
    dt, at = np.asarray(depth_t, np.float64), np.asarray(alpha_t, np.float64)
    p = d.shape[0]
    # The clamp decides which rays pass a gradient; that decision is taken on the single-
    # precision outputs against the single-precision bounds, as the renderer does.
    lo, hi = float(np.float32(1e-6)), float(np.float32(1.0 - 1e-6))
    ac = np.clip(a, lo, hi)
    inside = (a >= lo) & (a <= hi)
    per_ray = -(at * np.log(ac) + (1 - at) * np.log(1 - ac)) + w_depth * at * np.abs(d - dt)
    g_alpha = np.where(inside, -(at / ac) + (1 - at) / (1 - ac), 0.0) / p
    g_depth = w_depth * at * np.sign(d - dt) / p
    g_flow = None
    if flow is not None:
        df = np.asarray(flow, np.float64) - np.asarray(flow_t, np.float64)
        if flow_norm == 1:
            per_ray = per_ray + w_flow * at * np.abs(df).sum(axis=1)
            g_flow = w_flow * at[:, None] * np.sign(df) / p
        else:
            per_ray = per_ray + w_flow * at * (df * df).sum(axis=1)
            g_flow = 2.0 * w_flow * at[:, None] * df / p
    g_color = None
    if color is not None:
        dc = np.asarray(color, np.float64) - np.asarray(color_t, np.float64)
        per_ray = per_ray + w_color * at * np.abs(dc).sum(axis=1)
        g_color = w_color * at[:, None] * np.sign(dc) / p
    return float(per_ray.sum() / p), {"depth": g_depth, "alpha": g_alpha, "flow": g_flow, "color": g_color}
