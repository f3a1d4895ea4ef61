"""Seeded synthetic workloads for the two-parameter Fuzzy-Metaballs renderer.

Everything here is input construction: Gaussians (means, packed upper-triangular
precision factors, linear weights), pinhole cameras and random cotangents.  The
draws follow the five benchmark workloads of the renderer:

  fwd64      1 scene, N=40, one 64x64 view, forward only (depth, alpha, normals)
  fwdbwd128  1 scene, N=40, 20 views of 128x128 on a sphere, forward+backward
  batch16    16 scenes, N~U{10..100}, V~U{4..32}, 64^2/128^2/256^2 each, fwd+bwd
  flow480    1 scene, N=100, 8 pose pairs of 480x640, flow + depth + alpha, fwd+bwd
  large1080  1 scene, N=10000 in 50 clusters, one 1080x1920 view, fwd+bwd

Conventions (shared with the C ABI):
  * A Gaussian is (mu, U, lambda): the precision is Sigma^-1 = U^T U with U upper
    triangular, packed as (U00, U01, U02, U11, U12, U22); lambda > 0 is linear.
  * Cameras are world-to-camera [R|T] (x_cam = R x_world + T), OpenCV axes
    (x right, y down, z forward), intrinsics (fx, fy, cx, cy), pixel (row i, col j)
    has its centre at (j + 1/2, i + 1/2).
  * Rays are ordered view-major, then row-major within a view.

All arrays are float32 (int32 for sizes) exactly as both the GPU path and the
oracle consume them; the oracle upcasts the float32 values to float64.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Blend parameters beta1, beta2 that the paper reuses when rendering converted
# 3DGS scenes with the two-parameter weights (Interoperability section).
BETA1 = 21.4
BETA2 = 3.14
# Shape scale eta of Eq. (7): the paper leaves it free; 1 for unit-scale scenes.
ETA = 1.0

_CONFIGS = ("fwd64", "fwdbwd128", "batch16", "flow480", "large1080")


def config_names():
    return _CONFIGS


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Scene:
    means: np.ndarray    # [N,3] float32
    prec: np.ndarray     # [N,6] float32, packed upper-triangular U
    weights: np.ndarray  # [N] float32, lambda > 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.prec.copy(), self.weights.copy())


@dataclass
class Cameras:
    w2c: np.ndarray                     # [V,3,4] float32
    intr: np.ndarray                    # [V,4] float32 (fx, fy, cx, cy)
    hw: np.ndarray                      # [V,2] int32 (H, W)
    w2c_b: Optional[np.ndarray] = None  # [V,3,4] second pose (flow target) or None
    intr_b: Optional[np.ndarray] = None  # [V,4] or None
    w2c_c: Optional[np.ndarray] = None  # [V,3,4] optional third pose (backward-flow target)
    intr_c: Optional[np.ndarray] = None  # [V,4] or None

    @property
    def v(self) -> int:
        return int(self.w2c.shape[0])

    @property
    def n_rays(self) -> int:
        return int(np.sum(self.hw[:, 0].astype(np.int64) * self.hw[:, 1]))

    @property
    def has_flow(self) -> bool:
        return self.w2c_b is not None


@dataclass
class Workload:
    name: str
    scenes: List[Scene]
    cameras: List[Cameras]
    targets: List[Scene]          # perturbed copies the loss targets are rendered from
    betas: np.ndarray             # [2] float32
    eta: float
    normals: bool = True          # render per-ray normals
    backward: bool = True         # forward+backward workload
    loss: str = "depth_l1_bce"    # "depth_l1_bce" or "flow_l2"
    notes: dict = field(default_factory=dict)

    @property
    def n_rays(self) -> int:
        return sum(c.n_rays for c in self.cameras)

    @property
    def n_pairs(self) -> int:
        return sum(s.n * c.n_rays for s, c in zip(self.scenes, self.cameras))


# ----------------------------------------------------------------------------------------
# Gaussians
# ----------------------------------------------------------------------------------------

def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z) [N,4] -> rotation matrices [N,3,3] (float64)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((q.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - w * z)
    r[:, 0, 2] = 2 * (x * z + w * y)
    r[:, 1, 0] = 2 * (x * y + w * z)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - w * x)
    r[:, 2, 0] = 2 * (x * z - w * y)
    r[:, 2, 1] = 2 * (y * z + w * x)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def packed_upper_from_cov(rot: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Covariance R diag(s^2) R^T -> packed upper-triangular U with U^T U = Sigma^-1.

    Sigma^-1 = R diag(s^-2) R^T is formed in float64 and factored by Cholesky
    (Sigma^-1 = L L^T, U = L^T, positive diagonal).
    """
    prec = rot @ (np.einsum("nk,njk->njk", scales ** -2.0, rot)).transpose(0, 2, 1)
    prec = 0.5 * (prec + prec.transpose(0, 2, 1))
    lo = np.linalg.cholesky(prec)
    u = lo.transpose(0, 2, 1)
    return np.stack([u[:, 0, 0], u[:, 0, 1], u[:, 0, 2], u[:, 1, 1], u[:, 1, 2], u[:, 2, 2]], axis=1)


def make_scene(g: np.random.Generator, n: int, means: np.ndarray,
               log_s_range=(0.05, 0.2), w_range=(0.5, 1.0)) -> Scene:
    """Draw log-scales, rotations and weights for `n` Gaussians at the given means.

    Draw order per block: (means by the caller), log-scales, quaternions, weights.
    """
    lo, hi = math.log(log_s_range[0]), math.log(log_s_range[1])
    scales = np.exp(g.uniform(lo, hi, size=(n, 3)))
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rot = _quat_to_rot(q)
    w = g.uniform(w_range[0], w_range[1], size=n)
    prec = packed_upper_from_cov(rot, scales)
    return Scene(means.astype(np.float32), prec.astype(np.float32), w.astype(np.float32))


def _uniform_scene(g: np.random.Generator, n: int) -> Scene:
    means = g.uniform(-1.0, 1.0, size=(n, 3))
    return make_scene(g, n, means)


def _cluster_scene(g: np.random.Generator, n: int, k: int = 50, sigma: float = 0.1) -> Scene:
    centres = g.uniform(-1.0, 1.0, size=(k, 3))
    which = g.integers(0, k, size=n)
    means = centres[which] + sigma * g.standard_normal((n, 3))
    return make_scene(g, n, means, log_s_range=(0.005, 0.05))


def perturb_means(scene: Scene, g: np.random.Generator, sigma: float = 0.02) -> Scene:
    out = scene.copy()
    out.means = (scene.means.astype(np.float64)
                 + sigma * g.standard_normal(scene.means.shape)).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------
# Cameras
# ----------------------------------------------------------------------------------------

def look_at(centre, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World-to-camera [R|T] (OpenCV axes) for a camera at `centre` looking at `target`."""
    c = np.asarray(centre, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    u = np.asarray(up, dtype=np.float64)
    if abs(float(z @ u)) > 0.99:
        u = np.array([0.0, 1.0, 0.0])
    y = -u + (u @ z) * z
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    r = np.stack([x, y, z])
    return np.concatenate([r, (-r @ c)[:, None]], axis=1)


def fibonacci_sphere(n: int, radius: float = 3.0) -> np.ndarray:
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)


def _intr(h: int, w: int, f: Optional[float] = None) -> np.ndarray:
    f = float(h) if f is None else f
    return np.array([f, f, w / 2.0, h / 2.0])


def _front_camera(h: int, w: int) -> Cameras:
    """One camera at (0,0,-3) with R = I (looking along +z at the origin), fx = fy = H."""
    e = np.concatenate([np.eye(3), np.array([[0.0], [0.0], [3.0]])], axis=1)
    return Cameras(e[None].astype(np.float32), _intr(h, w)[None].astype(np.float32),
                   np.array([[h, w]], dtype=np.int32))


def _sphere_cameras(v: int, h: int, w: int) -> Cameras:
    cs = fibonacci_sphere(v)
    e = np.stack([look_at(c) for c in cs])
    intr = np.tile(_intr(h, w), (v, 1))
    return Cameras(e.astype(np.float32), intr.astype(np.float32),
                   np.tile(np.array([h, w], dtype=np.int32), (v, 1)))


def _axis_angle(axis: np.ndarray, ang: float) -> np.ndarray:
    a = axis / np.linalg.norm(axis)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * (k @ k)


def _perturbed_pose(g: np.random.Generator, r: np.ndarray, c: np.ndarray, rot_sigma_deg: float,
                    trans_sigma: float) -> np.ndarray:
    """World-to-camera [3,4] of a pose near (rotation r, centre c): the camera-to-world rotation
    premultiplied by a rotation of N(0, rot_sigma_deg^2) degrees about a uniformly random axis
    (about the camera centre), the centre moved by N(0, trans_sigma^2 I)."""
    axis = g.standard_normal(3)
    ang = math.radians(rot_sigma_deg) * g.standard_normal()
    r_b = (_axis_angle(axis, ang) @ r.T).T
    c_b = c + trans_sigma * g.standard_normal(3)
    return np.concatenate([r_b, (-r_b @ c_b)[:, None]], axis=1)


def with_backward_flow(cams: Cameras, seed: int, rot_sigma_deg: float = 2.0,
                       trans_sigma: float = 0.05) -> Cameras:
    """Copy of a flow camera set with a third pose per view (the previous frame, for backward
    flow), drawn with the same recipe as the second pose from its own seeded stream."""
    if cams.w2c_b is None:
        raise ValueError("backward flow needs a camera set that already has a second pose")
    g = _rng(seed)
    ec = []
    for e in cams.w2c.astype(np.float64):
        ec.append(_perturbed_pose(g, e[:, :3], -e[:, :3].T @ e[:, 3], rot_sigma_deg, trans_sigma))
    return Cameras(cams.w2c, cams.intr, cams.hw, cams.w2c_b, cams.intr_b,
                   np.stack(ec).astype(np.float32), cams.intr.copy())


def _flow_cameras(g: np.random.Generator, v: int, h: int, w: int,
                  rot_sigma_deg: float = 2.0, trans_sigma: float = 0.05) -> Cameras:
    """First poses look at the origin from directions uniform on the sphere (radius 3).

    The second pose premultiplies the camera-to-world rotation by a rotation of
    N(0, rot_sigma_deg^2) degrees about a uniformly random axis (about the camera
    centre) and moves the centre by N(0, trans_sigma^2 I).
    """
    dirs = g.standard_normal((v, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ea, eb = [], []
    for k in range(v):
        c = 3.0 * dirs[k]
        e = look_at(c)
        ea.append(e)
        eb.append(_perturbed_pose(g, e[:, :3], c, rot_sigma_deg, trans_sigma))
    intr = np.tile(_intr(h, w), (v, 1)).astype(np.float32)
    return Cameras(np.stack(ea).astype(np.float32), intr,
                   np.tile(np.array([h, w], dtype=np.int32), (v, 1)),
                   np.stack(eb).astype(np.float32), intr.copy())


# ----------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------

def make_config(name: str, seed: Optional[int] = None) -> Workload:
    """Build one of the five named workloads (seeded; default seeds 1..5)."""
    if name not in _CONFIGS:
        raise ValueError(f"unknown workload {name!r}; one of {_CONFIGS}")
    idx = _CONFIGS.index(name)
    seed = idx + 1 if seed is None else seed
    g = _rng(seed)
    gp = _rng(seed + 1000)
    betas = np.array([BETA1, BETA2], dtype=np.float32)
    if name == "fwd64":
        s = _uniform_scene(g, 40)
        return Workload(name, [s], [_front_camera(64, 64)], [perturb_means(s, gp)], betas, ETA,
                        normals=True, backward=False)
    if name == "fwdbwd128":
        s = _uniform_scene(g, 40)
        return Workload(name, [s], [_sphere_cameras(20, 128, 128)], [perturb_means(s, gp)],
                        betas, ETA, normals=True, backward=True)
    if name == "batch16":
        ns = g.integers(10, 101, size=16)
        vs = g.integers(4, 33, size=16)
        res = g.choice(np.array([64, 128, 256]), size=16)
        scenes = [_uniform_scene(g, int(n)) for n in ns]
        cams = [_sphere_cameras(int(v), int(r), int(r)) for v, r in zip(vs, res)]
        targets = [perturb_means(s, gp) for s in scenes]
        return Workload(name, scenes, cams, targets, betas, ETA, normals=True, backward=True)
    if name == "flow480":
        s = _uniform_scene(g, 100)
        cams = _flow_cameras(g, 8, 480, 640)
        return Workload(name, [s], [cams], [perturb_means(s, gp)], betas, ETA,
                        normals=False, backward=True, loss="flow_l2")
    # large1080
    s = _cluster_scene(g, 10000)
    return Workload(name, [s], [_front_camera(1080, 1920)], [perturb_means(s, gp)], betas, ETA,
                    normals=True, backward=True)


def pixel_indices(cams: Cameras, rays: Optional[np.ndarray] = None):
    """(view, row, col) int32 arrays for global ray indices (default: all rays)."""
    hw = cams.hw.astype(np.int64)
    counts = hw[:, 0] * hw[:, 1]
    off = np.concatenate([[0], np.cumsum(counts)])
    if rays is None:
        rays = np.arange(off[-1], dtype=np.int64)
    rays = np.asarray(rays, dtype=np.int64)
    view = np.searchsorted(off, rays, side="right") - 1
    local = rays - off[view]
    w = hw[view, 1]
    return view.astype(np.int32), (local // w).astype(np.int32), (local % w).astype(np.int32)


def random_cotangents(n_rays: int, seed: int, flow: bool = True, normals: bool = True):
    """Seeded standard-normal cotangents for depth, alpha, normals [P,3] and flow [P,2]."""
    g = _rng(seed)
    out = {"depth": g.standard_normal(n_rays).astype(np.float32),
           "alpha": g.standard_normal(n_rays).astype(np.float32)}
    out["normal"] = g.standard_normal((n_rays, 3)).astype(np.float32) if normals else None
    out["flow"] = g.standard_normal((n_rays, 2)).astype(np.float32) if flow else None
    return out
