"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each `pin_*` function raises AssertionError when the oracle disagrees with:
closed forms (single isotropic Gaussian, two-Gaussian blend), a brute-force line
search of the density along the ray built from the covariance (not from the
factor U), the converted-3DGS alpha the paper's Interoperability section implies,
algebraic identities of Eq. (8), invariances (permutation, scale with eta,
rigid motion), the rotation homography and translation parallax of the flow,
and central finite differences of the oracle's own forward pass for every
gradient.  The same functions run against deliberately broken copies of the
oracle (tests/test_oracle_mutants.py) to show that each plausible slip fails at
least one pin.
"""

from __future__ import annotations

import math
import os

import numpy as np

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

B1, B2 = 21.4, 3.14


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _unit(x):
    x = np.asarray(x, dtype=np.float64)
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _rot(g):
    q = _unit(g.standard_normal(4))
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _cov_and_packed(g, smin=0.05, smax=0.3):
    """Random covariance Sigma = R diag(s^2) R^T and the packed upper factor of Sigma^-1."""
    r = _rot(g)
    s = np.exp(g.uniform(math.log(smin), math.log(smax), 3))
    cov = r @ np.diag(s ** 2) @ r.T
    lo = np.linalg.cholesky(np.linalg.inv(cov))
    u = lo.T
    return cov, np.array([u[0, 0], u[0, 1], u[0, 2], u[1, 1], u[1, 2], u[2, 2]])


def _packed_iso(s):
    return np.array([1 / s, 0, 0, 1 / s, 0, 1 / s])


def _scene(means, prec, weights, betas=(B1, B2), eta=1.0):
    return O.OracleScene.of(np.asarray(means), np.asarray(prec), np.asarray(weights),
                            np.asarray(betas, dtype=np.float64), eta)


def _random_scene(g, n, spread=0.6, betas=(B1, B2), eta=1.0):
    means = g.uniform(-spread, spread, (n, 3))
    covs, prec = zip(*[_cov_and_packed(g) for _ in range(n)])
    w = g.uniform(0.5, 1.5, n)
    return _scene(means, np.array(prec), w, betas, eta), np.array(covs)


def _rays_at(g, targets, o, jitter=0.15):
    """Unit rays from origin o aimed near the given points."""
    aim = targets + jitter * g.standard_normal(targets.shape)
    return np.tile(o, (len(aim), 1)), _unit(aim - o)


def _close(a, b, rtol, atol, what):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    err = np.abs(a - b)
    lim = atol + rtol * np.abs(b)
    assert np.all(err <= lim), f"{what}: max err {err.max():.3e} (worst excess {np.max(err - lim):.3e})"


# ---------------------------------------------------------------------------------------
# Eq. (2), (4), (8), (17): single Gaussians
# ---------------------------------------------------------------------------------------

def pin_isotropic_closed_form():
    """U = I/s: t = (mu-o).v, m = |o+tv-mu|^2/s^2, n = (o+tv-mu)/|.|, alpha = 1-exp(-lam e^{-m/2})."""
    g = _rng(11)
    for _ in range(20):
        mu = g.uniform(-1, 1, 3)
        s = g.uniform(0.05, 0.5)
        lam = g.uniform(0.2, 3.0)
        o = g.uniform(-4, 4, 3)
        v = _unit(mu + 0.3 * g.standard_normal(3) - o)
        sc = _scene(mu[None], _packed_iso(s)[None], [lam])
        t, d, z, nrm = O.ray_terms(sc, o, v)
        t_ref = (mu - o) @ v
        x = o + t_ref * v - mu
        m_ref = (x @ x) / s ** 2
        _close(t[0], t_ref, 1e-12, 1e-12, "isotropic t")
        _close(d[0], math.log(lam) - 0.5 * m_ref, 1e-12, 1e-12, "isotropic d")
        _close(z[0], B1 * d[0] - B2 * t_ref, 1e-12, 1e-12, "isotropic z")
        _close(nrm[0], x / np.linalg.norm(x), 1e-9, 1e-9, "isotropic normal")
        out = O.render(sc, o[None], v[None])
        _close(out["depth"][0], t_ref, 1e-12, 1e-12, "N=1 depth")
        _close(out["alpha"][0], 1 - math.exp(-lam * math.exp(-0.5 * m_ref)), 1e-12, 1e-14,
               "N=1 alpha")
        _close(out["normal"][0], x / np.linalg.norm(x), 1e-9, 1e-9, "N=1 normal")


def _maha_cov(cov, mu, x):
    dx = x - mu
    return float(dx @ np.linalg.solve(cov, dx))


def _golden_max(f, lo, hi, iters=200):
    gr = (math.sqrt(5) - 1) / 2
    a, b = lo, hi
    c, d = b - gr * (b - a), a + gr * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - gr * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + gr * (b - a)
            fd = f(d)
    return 0.5 * (a + b)


def pin_bruteforce_peak():
    """Anisotropic Gaussians: the oracle's t_i and d_i equal a golden-section maximisation
    of log(lambda) - 1/2 (x-mu)^T Sigma^-1 (x-mu) along the ray, with Sigma^-1 applied by
    solving against the covariance; its n_i is the direction of the finite-difference
    gradient of that Mahalanobis form at the peak (Eq. 17)."""
    g = _rng(12)
    for _ in range(25):
        cov, prec = _cov_and_packed(g)
        mu = g.uniform(-1, 1, 3)
        lam = g.uniform(0.3, 2.0)
        o = g.uniform(-4, 4, 3)
        v = _unit(mu + 0.2 * g.standard_normal(3) - o)
        sc = _scene(mu[None], prec[None], [lam])
        t, d, _, nrm = O.ray_terms(sc, o, v)
        f = lambda tt: math.log(lam) - 0.5 * _maha_cov(cov, mu, o + tt * v)  # noqa: E731
        grid = np.linspace(-10, 10, 4001)
        k = int(np.argmax([f(tt) for tt in grid]))
        tb = _golden_max(f, grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)])
        _close(t[0], tb, 0, 2e-7, "peak depth vs line search")
        _close(d[0], f(tb), 1e-10, 1e-10, "peak log-density vs line search")
        x = o + tb * v
        h = 1e-6
        grad = np.array([(_maha_cov(cov, mu, x + h * e) - _maha_cov(cov, mu, x - h * e)) / (2 * h)
                         for e in np.eye(3)])
        _close(nrm[0], _unit(grad), 0, 2e-6, "normal vs gradient of the Mahalanobis form")
        # optimality: the normal is perpendicular to the ray at the peak
        assert abs(nrm[0] @ v) < 1e-9, "n_i . v != 0 at the peak"


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, val = line.split("=", 1)
            vals[k.strip()] = val.strip()
    return vals


def pin_interop_alpha():
    """A converted 3DGS Gaussian has lambda = log 80; a ray through its mean renders alpha = 79/80
    whatever its shape (Interoperability section with Eq. 8)."""
    gold = read_golden("interop_alpha.txt")
    lam = eval(gold["lambda"], {"log": math.log})  # noqa: S307 (fixture is ours)
    alpha_ref = eval(gold["alpha"], {})  # noqa: S307
    g = _rng(13)
    for _ in range(10):
        _, prec = _cov_and_packed(g)
        mu = g.uniform(-1, 1, 3)
        o = g.uniform(-4, 4, 3)
        v = _unit(mu - o)
        out = O.render(_scene(mu[None], prec[None], [lam]), o[None], v[None])
        _close(out["alpha"][0], alpha_ref, 0, 1e-12, "alpha through the mean")
        _close(out["depth"][0], np.linalg.norm(mu - o), 1e-10, 1e-10, "depth at the mean")


def pin_alpha_identities():
    """Eq. (8): 1 - alpha(A u B) = (1 - alpha(A)) (1 - alpha(B)); alpha in [0,1]; monotone in lambda."""
    g = _rng(14)
    sc, _ = _random_scene(g, 6)
    o = np.array([0.0, 0.0, -3.0])
    orig, dirs = _rays_at(g, sc.means, o)
    a_all = O.render(sc, orig, dirs)["alpha"]
    part = lambda idx: _scene(sc.means[idx], sc.prec[idx], sc.weights[idx])  # noqa: E731
    a1 = O.render(part([0, 1, 2]), orig, dirs)["alpha"]
    a2 = O.render(part([3, 4, 5]), orig, dirs)["alpha"]
    _close(1 - a_all, (1 - a1) * (1 - a2), 1e-12, 1e-15, "alpha union")
    assert np.all((a_all >= 0) & (a_all <= 1))
    heavier = _scene(sc.means, sc.prec, sc.weights * np.array([1, 1, 1.5, 1, 1, 1]))
    assert np.all(O.render(heavier, orig, dirs)["alpha"] >= a_all)


# ---------------------------------------------------------------------------------------
# Eq. (3), (7): blending
# ---------------------------------------------------------------------------------------

def _single_terms(sc, i, orig, dirs):
    one = _scene(sc.means[[i]], sc.prec[[i]], sc.weights[[i]], sc.betas, sc.eta)
    out = O.render(one, orig, dirs)
    dens = -np.log1p(-out["alpha"])      # sum of delta = delta_i for N = 1
    return out["depth"], np.log(dens), out["normal"]


def pin_two_gaussian_blend():
    """N = 2: t_f = t_2 + (t_1 - t_2) sigma(z_1 - z_2), z_i = beta1 d_i - (beta2/eta) t_i, with t_i, d_i,
    n_i taken from one-Gaussian renders; the blended normal is the same convex combination, normalised."""
    g = _rng(15)
    for eta in (1.0, 2.5):
        sc, _ = _random_scene(g, 2, spread=0.3, eta=eta)
        o = np.array([0.3, -0.2, -3.0])
        orig, dirs = _rays_at(g, np.repeat(sc.means, 4, axis=0), o, jitter=0.05)
        t1, d1, n1 = _single_terms(sc, 0, orig, dirs)
        t2, d2, n2 = _single_terms(sc, 1, orig, dirs)
        z1, z2 = B1 * d1 - B2 / eta * t1, B1 * d2 - B2 / eta * t2
        s = 1 / (1 + np.exp(-(z1 - z2)))
        out = O.render(sc, orig, dirs)
        _close(out["depth"], t2 + (t1 - t2) * s, 1e-9, 1e-9, "two-Gaussian depth blend")
        nb = s[:, None] * n1 + (1 - s)[:, None] * n2
        _close(out["normal"], _unit(nb), 1e-7, 1e-7, "two-Gaussian normal blend")


def pin_zero_betas_mean():
    """beta1 = beta2 = 0 makes every weight equal: t_f is the plain mean of the t_i."""
    g = _rng(16)
    sc, _ = _random_scene(g, 7, betas=(0.0, 0.0))
    o = np.array([0.1, 0.2, -3.0])
    orig, dirs = _rays_at(g, sc.means, o)
    out = O.render(sc, orig, dirs)
    for r in range(len(orig)):
        ts = [_single_terms(sc, i, orig[[r]], dirs[[r]])[0][0] for i in range(sc.n)]
        _close(out["depth"][r], np.mean(ts), 1e-10, 1e-10, "zero-beta mean depth")


def pin_permutation():
    g = _rng(17)
    sc, _ = _random_scene(g, 9)
    o = np.array([0.0, 0.0, -3.0])
    orig, dirs = _rays_at(g, sc.means, o)
    ref = O.render(sc, orig, dirs)
    perm = g.permutation(sc.n)
    out = O.render(_scene(sc.means[perm], sc.prec[perm], sc.weights[perm]), orig, dirs)
    for k in ("depth", "alpha", "normal"):
        _close(out[k], ref[k], 1e-10, 1e-12, f"permutation {k}")


# ---------------------------------------------------------------------------------------
# Cameras, rays and flow (Sec. 5)
# ---------------------------------------------------------------------------------------

def _look_at(c, target=(0, 0, 0)):
    z = _unit(np.asarray(target, float) - c)
    u = np.array([0.0, 0.0, 1.0])
    y = _unit(-u + (u @ z) * z)
    x = np.cross(y, z)
    r = np.stack([x, y, z])
    return np.concatenate([r, (-r @ c)[:, None]], axis=1)


def pin_pixel_ray_hand_case():
    """Camera at (0,0,-3), R = I, fx = fy = 64, cx = cy = 32: pixel (row 0, col 63) has the
    camera-frame direction (31.5/64, -31.5/64, 1), normalised."""
    e = np.array([[1.0, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 3]])
    k = np.array([64.0, 64.0, 32.0, 32.0])
    o, v = O.pixel_rays([0], [0], [63], e[None], k[None])
    _close(o[0], [0, 0, -3], 0, 1e-15, "camera centre")
    _close(v[0], _unit([31.5 / 64, -31.5 / 64, 1.0]), 0, 1e-15, "pixel direction")
    uv = O.project([0], (o[0] + 2.7 * v[0])[None], e[None], k[None])
    _close(uv[0], [63.5, 0.5], 0, 1e-12, "projection of a point on the pixel ray")


def pin_rays_reproject():
    """Points on the ray of pixel (i, j) project back onto the pixel centre (j + 1/2, i + 1/2)."""
    g = _rng(18)
    e = np.stack([_look_at(3 * _unit(g.standard_normal(3))) for _ in range(3)])
    k = np.array([[80.0, 90.0, 40.0, 30.0], [64, 64, 32, 32], [100, 100, 60, 45]])
    view = np.repeat(np.arange(3), 5).astype(np.int32)
    row = g.integers(0, 60, 15).astype(np.int32)
    col = g.integers(0, 80, 15).astype(np.int32)
    o, v = O.pixel_rays(view, row, col, e, k)
    uv = O.project(view, o + g.uniform(0.5, 6, (15, 1)) * v, e, k)
    _close(uv, np.stack([col + 0.5, row + 0.5], axis=1), 0, 1e-10, "reprojection")


def pin_dir_rays():
    """Explicit-direction rays (the random ray minibatches of Sec. 4): every ray starts at the
    centre of its view's camera and has the unit direction of the given vector, whatever its
    length.  Hand cases on an axis-aligned camera, then pixel-centre directions of rotated cameras
    (formed here from R^T d_c, independently of the oracle) scaled by random positive factors,
    which must give exactly the pixel rays' origins and unit directions."""
    e = np.array([[1.0, 0, 0, -1], [0, 1, 0, -2], [0, 0, 1, 3]])  # R = I, centre (1, 2, -3)
    o, v = O.dir_rays([0, 0, 0], [[0, 0, 7.5], [3, 4, 0], [0, -1e-3, 0]], e[None])
    _close(o, np.tile([1.0, 2.0, -3.0], (3, 1)), 0, 1e-15, "camera centre")
    _close(v, [[0, 0, 1], [0.6, 0.8, 0], [0, -1, 0]], 0, 1e-15, "unit direction")
    g = _rng(23)
    es = np.stack([_look_at(3 * _unit(g.standard_normal(3))) for _ in range(3)])
    ks = np.array([[80.0, 90.0, 40.0, 30.0], [64, 64, 32, 32], [100, 100, 60, 45]])
    view = np.repeat(np.arange(3), 6).astype(np.int32)
    row = g.integers(0, 60, 18).astype(np.int32)
    col = g.integers(0, 80, 18).astype(np.int32)
    dc = np.stack([(col + 0.5 - ks[view, 2]) / ks[view, 0], (row + 0.5 - ks[view, 3]) / ks[view, 1],
                   np.ones(18)], axis=1)
    d = np.einsum("pji,pj->pi", es[view, :, :3], dc)  # R^T d_c per ray
    scale = np.exp(g.uniform(-3.0, 3.0, (18, 1)))
    o, v = O.dir_rays(view, d * scale, es)
    op, vp = O.pixel_rays(view, row, col, es, ks)
    centres = -np.einsum("kji,kj->ki", es[:, :, :3], es[:, :, 3])
    _close(o, centres[view], 0, 1e-14, "origin = camera centre of the ray's view")
    _close(o, op, 0, 1e-15, "origins of explicit and pixel rays")
    _close(np.linalg.norm(v, axis=1), np.ones(18), 0, 1e-15, "unit length")
    _close(v, vp, 0, 1e-15, "directions of explicit and pixel rays")


def _flow_setup(g, n=6):
    sc, _ = _random_scene(g, n, spread=0.5)
    c = np.array([0.4, -2.6, 1.2])
    ea = _look_at(c)
    k = np.array([60.0, 60.0, 40.0, 30.0])
    view = np.zeros(24, dtype=np.int32)
    row = g.integers(0, 60, 24).astype(np.int32)
    col = g.integers(0, 80, 24).astype(np.int32)
    o, v = O.pixel_rays(view, row, col, ea[None], k[None])
    return sc, ea, k, view, row, col, o, v


def pin_flow_equal_poses():
    g = _rng(19)
    sc, ea, k, view, row, col, o, v = _flow_setup(g)
    out = O.render(sc, o, v, view=view, w2c_a=ea[None], intr_a=k[None], w2c_b=ea[None], intr_b=k[None])
    assert np.all(out["flow"] == 0.0), "flow must vanish for equal poses"


def pin_flow_rotation_homography():
    """Second pose rotated about the camera centre (R_B = Q R_A, T_B = Q T_A): the flow of pixel
    (i, j) is the homography K Q K^-1 (j+1/2, i+1/2, 1) minus the pixel, whatever the scene."""
    g = _rng(20)
    sc, ea, k, view, row, col, o, v = _flow_setup(g)
    axis = _unit(g.standard_normal(3))
    ang = math.radians(3.0)
    kx = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    q = np.eye(3) + math.sin(ang) * kx + (1 - math.cos(ang)) * kx @ kx
    eb = np.concatenate([q @ ea[:, :3], (q @ ea[:, 3])[:, None]], axis=1)
    out = O.render(sc, o, v, view=view, w2c_a=ea[None], intr_a=k[None], w2c_b=eb[None], intr_b=k[None])
    kk = np.array([[k[0], 0, k[2]], [0, k[1], k[3]], [0, 0, 1]])
    hom = kk @ q @ np.linalg.inv(kk)
    px = np.stack([col + 0.5, row + 0.5, np.ones(len(col))], axis=0)
    hp = hom @ px
    ref = (hp[:2] / hp[2]).T - px[:2].T
    _close(out["flow"], ref, 1e-9, 1e-9, "rotation homography flow")


def pin_flow_translation():
    """Second pose translated by c (same R): q_B = t_f * d_cam/|d_cam| - R c, projected with K, minus
    the pixel; d_cam = ((j+1/2-cx)/fx, (i+1/2-cy)/fy, 1) is the pixel's camera-frame direction."""
    g = _rng(21)
    sc, ea, k, view, row, col, o, v = _flow_setup(g)
    shift = np.array([0.05, -0.08, 0.03])
    eb = ea.copy()
    eb[:, 3] = ea[:, 3] - ea[:, :3] @ shift
    out = O.render(sc, o, v, view=view, w2c_a=ea[None], intr_a=k[None], w2c_b=eb[None], intr_b=k[None])
    dc = np.stack([(col + 0.5 - k[2]) / k[0], (row + 0.5 - k[3]) / k[1], np.ones(len(col))], axis=1)
    qa = out["depth"][:, None] * _unit(dc)
    qb = qa - (ea[:, :3] @ shift)[None]
    ref = np.stack([k[0] * qb[:, 0] / qb[:, 2] + k[2], k[1] * qb[:, 1] / qb[:, 2] + k[3]], axis=1)
    ref -= np.stack([col + 0.5, row + 0.5], axis=1)
    _close(out["flow"], ref, 1e-9, 1e-9, "translation flow")


def pin_flow_both_directions():
    """Forward and backward flow (Sec. 5): with the third pose translated by -c when the second is
    translated by +c, both follow the translation parallax formula with their own shift; with the
    third pose equal to the first, the backward columns are exactly zero; and the gradient of a
    4-column flow objective matches central differences."""
    g = _rng(30)
    sc, ea, k, view, row, col, o, v = _flow_setup(g)
    shift = np.array([0.05, -0.08, 0.03])
    eb, ec = ea.copy(), ea.copy()
    eb[:, 3] = ea[:, 3] - ea[:, :3] @ shift
    ec[:, 3] = ea[:, 3] + ea[:, :3] @ shift
    cam = dict(view=view, w2c_a=ea[None], intr_a=k[None], w2c_b=eb[None], intr_b=k[None],
               w2c_c=ec[None], intr_c=k[None])
    out = O.render(sc, o, v, **cam)
    assert out["flow"].shape == (len(o), 4)
    dc = np.stack([(col + 0.5 - k[2]) / k[0], (row + 0.5 - k[3]) / k[1], np.ones(len(col))], axis=1)
    qa = out["depth"][:, None] * _unit(dc)
    px = np.stack([col + 0.5, row + 0.5], axis=1)
    for cols, sgn in ((slice(0, 2), 1.0), (slice(2, 4), -1.0)):
        qx = qa - sgn * (ea[:, :3] @ shift)[None]
        ref = np.stack([k[0] * qx[:, 0] / qx[:, 2] + k[2], k[1] * qx[:, 1] / qx[:, 2] + k[3]], axis=1)
        _close(out["flow"][:, cols], ref - px, 1e-9, 1e-9, f"two-way translation flow {cols}")
    same = O.render(sc, o, v, **dict(cam, w2c_c=ea[None]))
    assert np.all(same["flow"][:, 2:] == 0.0), "backward flow to the first pose must vanish"
    _close(same["flow"][:, :2], out["flow"][:, :2], 0.0, 0.0, "forward flow independent of pose C")
    # gradient of sum(cot . flow4) through means, against central differences
    o8, v8, cam8 = o[:6], v[:6], dict(cam, view=view[:6])
    cot = {"flow": g.standard_normal((6, 4))}
    an = O.backward(sc, o8, v8, cot, **cam8)
    base = sc.means.reshape(-1)
    fd = np.zeros_like(base)
    for j in range(base.size):
        x0 = base[j]
        h = 1e-6 * max(1.0, abs(x0))
        base[j] = x0 + h
        fp = float(np.sum(cot["flow"] * O.render(sc, o8, v8, **cam8)["flow"]))
        base[j] = x0 - h
        fm = float(np.sum(cot["flow"] * O.render(sc, o8, v8, **cam8)["flow"]))
        base[j] = x0
        fd[j] = (fp - fm) / (2 * h)
    scale = max(1.0, float(np.max(np.abs(fd))))
    _close(an["means"].reshape(-1), fd, 1e-6, 1e-6 * scale, "FD gradient of two-way flow")


def pin_max_weight():
    """Direct-intersection quality max_i w_i (Sec. 6): 1 for a single Gaussian; 1/K for K identical
    Gaussians; for two equal isotropic Gaussians centred on the ray at t_1 < t_2 (both d_i equal),
    sigma((beta2/eta)(t_2 - t_1)), the weight of the nearer one."""
    g = _rng(31)
    o = np.array([0.0, 0.0, -3.0])
    dirs = _unit(np.array([[0.0, 0.0, 1.0], [0.02, -0.01, 1.0], [-0.03, 0.02, 1.0]]))
    orig = np.tile(o, (len(dirs), 1))
    one = _scene([[0.0, 0.0, 0.0]], [_packed_iso(0.2)], [1.0])
    assert np.all(np.abs(O.max_weight(one, orig, dirs) - 1.0) <= 1e-15)
    for kk in (2, 3, 5):
        many = _scene(np.zeros((kk, 3)), np.tile(_packed_iso(0.2), (kk, 1)), np.ones(kk))
        _close(O.max_weight(many, orig, dirs), np.full(len(dirs), 1.0 / kk), 1e-14, 0.0, f"{kk} copies")
    for eta in (1.0, 2.0):
        gap = float(g.uniform(0.05, 0.4))
        pair = _scene([[0.0, 0.0, 0.0], [0.0, 0.0, gap]], np.tile(_packed_iso(0.25), (2, 1)),
                      [1.0, 1.0], eta=eta)
        q = O.max_weight(pair, orig[:1], dirs[:1])
        _close(q, [1.0 / (1.0 + math.exp(-B2 / eta * gap))], 1e-12, 0.0, "two on-axis Gaussians")


# ---------------------------------------------------------------------------------------
# Zero-parameter model: alpha compositing, Eq. (9)-(10)
# ---------------------------------------------------------------------------------------

def _single_t_delta_n(sc, orig, dirs):
    """Per-Gaussian (t_i, delta_i, n_i) of each ray from one-Gaussian renders: depth = t_i,
    delta_i = -log(1 - alpha_i) (Eq. 8 inverted), normal = n_i."""
    ts, ds, ns = [], [], []
    for i in range(sc.n):
        one = _scene(sc.means[[i]], sc.prec[[i]], sc.weights[[i]])
        out = O.render(one, orig, dirs)
        ts.append(out["depth"])
        ds.append(-np.log1p(-out["alpha"]))
        ns.append(out["normal"])
    return np.array(ts).T, np.array(ds).T, np.stack(ns, axis=1)


def _sorted_composite(t, delta, nrm):
    """Eq. (9)-(10) by sorting the intersections and multiplying transmittances front to back
    (the description of the paper's sort-based renderer), then Eq. (3)."""
    depth, normal = np.empty(len(t)), np.empty((len(t), 3))
    for r in range(len(t)):
        order = np.argsort(t[r], kind="stable")
        trans, wsum, tsum, nsum = 1.0, 0.0, 0.0, np.zeros(3)
        for i in order:
            w = trans * (1.0 - math.exp(-delta[r, i]))
            wsum += w
            tsum += w * t[r, i]
            nsum += w * nrm[r, i]
            trans *= math.exp(-delta[r, i])
        depth[r] = tsum / wsum
        normal[r] = nsum / np.linalg.norm(nsum)
    return depth, normal


def pin_composite_single_gaussian():
    """With one Gaussian the compositing weight is its own: depth t_1, the same alpha and normal
    as the two-parameter model."""
    g = _rng(40)
    sc, _ = _random_scene(g, 1, spread=0.2)
    orig, dirs = _rays_at(g, np.repeat(sc.means, 6, axis=0), np.array([0.2, 0.1, -3.0]), jitter=0.1)
    a, b = O.render(sc, orig, dirs), O.render(sc, orig, dirs, model="composite")
    for k in ("depth", "alpha", "normal"):
        _close(b[k], a[k], 1e-14, 1e-14, f"single-Gaussian composite {k}")


def pin_composite_sorted_reference():
    """Random scenes of up to 6 Gaussians: the oracle's unsorted strict-inequality sums match a
    front-to-back sort with running transmittance built from one-Gaussian renders."""
    g = _rng(41)
    for n in (2, 4, 6):
        sc, _ = _random_scene(g, n, spread=0.35)
        orig, dirs = _rays_at(g, np.repeat(sc.means, 3, axis=0), np.array([0.3, -0.2, -3.0]), jitter=0.08)
        t, delta, nrm = _single_t_delta_n(sc, orig, dirs)
        ref_d, ref_n = _sorted_composite(t, delta, nrm)
        out = O.render(sc, orig, dirs, model="composite")
        _close(out["depth"], ref_d, 1e-9, 1e-9, f"composite depth vs sorted (N={n})")
        _close(out["normal"], ref_n, 1e-8, 1e-8, f"composite normal vs sorted (N={n})")
        _close(out["alpha"], -np.expm1(-delta.sum(axis=1)), 1e-12, 1e-14, "composite alpha (Eq. 8)")


def pin_composite_ties():
    """Equal t_i do not attenuate one another (strict inequality of Eq. 10): three identical
    Gaussians behind a fourth on the ray axis each get T = exp(-delta_front)."""
    prec = np.tile(_packed_iso(0.2), (4, 1))
    means = np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.5], [0.0, 0.0, 0.5], [0.0, 0.0, 0.0]])
    sc = _scene(means, prec, [0.8, 0.8, 0.8, 0.6])
    orig = np.tile([0.0, 0.0, -3.0], (3, 1))
    dirs = _unit(np.array([[0.0, 0.0, 1.0], [0.01, 0.02, 1.0], [-0.02, 0.01, 1.0]]))
    t, delta, _ = _single_t_delta_n(sc, orig, dirs)
    wf = -np.expm1(-delta[:, 3])
    wb = np.exp(-delta[:, 3]) * -np.expm1(-delta[:, 0])
    ref = (wf * t[:, 3] + 3 * wb * t[:, 0]) / (wf + 3 * wb)
    out = O.render(sc, orig, dirs, model="composite")
    _close(out["depth"], ref, 1e-12, 1e-12, "composite with tied intersections")
    q = O.max_weight(sc, orig, dirs, model="composite")
    _close(q, np.maximum(wf, wb) / (wf + 3 * wb), 1e-12, 0.0, "composite max weight with ties")


def pin_composite_background():
    """A ray far from every Gaussian (all densities underflow): every T_i is 1 and the log
    opacity equals d_i, so the weights are softmax(d_i)."""
    g = _rng(42)
    covs = [_cov_and_packed(g, 0.03, 0.06)[1] for _ in range(5)]
    sc = _scene(g.uniform(-0.3, 0.3, (5, 3)), np.array(covs), g.uniform(0.5, 1.5, 5))
    orig = np.array([[0.0, 0.0, -3.0]])
    dirs = _unit(np.array([[1.0, 0.2, 0.05]]))
    t, d, _, _ = O.ray_terms(sc, orig[0], dirs[0])
    assert np.all(d < -700), "the test ray must miss every Gaussian by far"
    w = np.exp(d - d.max())
    out = O.render(sc, orig, dirs, model="composite")
    assert np.isfinite(out["depth"]).all()
    _close(out["depth"], [(w * t).sum() / w.sum()], 1e-12, 1e-12, "background composite depth")


def pin_composite_scale_invariance():
    """Scene and camera scaled by k: the zero-parameter model needs no eta; depth scales by k,
    alpha and normals are unchanged."""
    g = _rng(43)
    sc, _ = _random_scene(g, 6, spread=0.4)
    o = np.array([0.2, -0.3, -3.0])
    orig, dirs = _rays_at(g, np.repeat(sc.means, 2, axis=0), o, jitter=0.1)
    base = O.render(sc, orig, dirs, model="composite")
    k = 3.7
    big = _scene(sc.means * k, sc.prec / k, sc.weights)
    out = O.render(big, orig * k, dirs, model="composite")
    _close(out["depth"], base["depth"] * k, 1e-10, 1e-10, "composite depth scale")
    _close(out["alpha"], base["alpha"], 1e-12, 1e-12, "composite alpha scale")
    _close(out["normal"], base["normal"], 1e-9, 1e-9, "composite normal scale")


def pin_composite_gradients_fd():
    """Central differences of the composite forward match its adjoint for means, precision
    factors, weights and colours through every output; the beta gradient is zero."""
    g = _rng(44)
    sc, ea, kk, view, row, col, o, v = _flow_setup(g, n=5)
    view, o, v = view[:8], o[:8], v[:8]
    eb = _look_at(np.array([0.5, -2.5, 1.1]))
    cam = dict(view=view, w2c_a=ea[None], intr_a=kk[None], w2c_b=eb[None], intr_b=kk[None],
               model="composite")
    p = len(o)
    cot = {"depth": g.standard_normal(p), "alpha": g.standard_normal(p),
           "normal": g.standard_normal((p, 3)), "flow": g.standard_normal((p, 2)),
           "color": g.standard_normal((p, 3))}
    sc = O.OracleScene.of(sc.means, sc.prec, sc.weights * 3.0, (B1, B2), 1.0, g.standard_normal((sc.n, 3)))
    an = O.backward(sc, o, v, cot, **cam)
    assert np.all(an["betas"] == 0.0)
    for name in ("means", "prec", "weights", "colors"):
        base = getattr(sc, name)
        fd = np.zeros_like(base)
        flat, fdf = base.reshape(-1), fd.reshape(-1)
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            x0 = flat[j]
            flat[j] = x0 + h
            fp = _loss(sc, o, v, cam, cot)
            flat[j] = x0 - h
            fm = _loss(sc, o, v, cam, cot)
            flat[j] = x0
            fdf[j] = (fp - fm) / (2 * h)
        scale = max(1.0, float(np.max(np.abs(fd))))
        _close(an[name], fd, 1e-6, 1e-6 * scale, f"composite FD gradient {name}")


# ---------------------------------------------------------------------------------------
# Split statistic (Sec. 8)
# ---------------------------------------------------------------------------------------

def pin_split_statistic():
    """lbar_i = (1/M) sum_j L_j w_ji: the mean loss for one Gaussian; the weights of a ray sum to
    one, so sum_i lbar_i = mean(L) for both models; equal weights (zero betas) give mean(L)/N; two
    Gaussians follow the sigmoid of z_1 - z_2 (blend) and the front-to-back compositing weights
    built from one-Gaussian renders (composite)."""
    g = _rng(50)
    o = np.array([0.2, -0.1, -3.0])
    sc, _ = _random_scene(g, 5, spread=0.4)
    orig, dirs = _rays_at(g, np.repeat(sc.means, 4, axis=0), o, jitter=0.2)
    loss = g.uniform(0.0, 2.0, len(orig))
    one = _scene(sc.means[[2]], sc.prec[[2]], sc.weights[[2]])
    for model in ("blend", "composite"):
        _close(O.split_statistic(one, orig, dirs, loss, model), [loss.mean()], 1e-14, 0.0, f"one Gaussian {model}")
        _close([O.split_statistic(sc, orig, dirs, loss, model).sum()], [loss.mean()], 1e-12, 0.0,
               f"weights sum to one ({model})")
    flat = _scene(sc.means, sc.prec, sc.weights, betas=(0.0, 0.0))
    _close(O.split_statistic(flat, orig, dirs, loss), np.full(sc.n, loss.mean() / sc.n), 1e-12, 0.0,
           "zero betas")
    two = _scene(sc.means[:2], sc.prec[:2], sc.weights[:2])
    t1, d1, _ = _single_terms(two, 0, orig, dirs)
    t2, d2, _ = _single_terms(two, 1, orig, dirs)
    s1 = 1.0 / (1.0 + np.exp(-((B1 * d1 - B2 * t1) - (B1 * d2 - B2 * t2))))
    _close(O.split_statistic(two, orig, dirs, loss), [np.mean(loss * s1), np.mean(loss * (1 - s1))],
           1e-10, 1e-12, "two Gaussians (blend)")
    t, delta, _ = _single_t_delta_n(two, orig, dirs)
    w = np.empty_like(t)
    for r in range(len(t)):
        a, b = (0, 1) if t[r, 0] < t[r, 1] else (1, 0)
        w[r, a] = -math.expm1(-delta[r, a])
        w[r, b] = math.exp(-delta[r, a]) * -math.expm1(-delta[r, b])
    w /= w.sum(axis=1, keepdims=True)
    _close(O.split_statistic(two, orig, dirs, loss, "composite"), (loss[:, None] * w).mean(axis=0), 1e-10,
           1e-12, "two Gaussians (composite)")


def _cov_of_packed(u):
    U = np.array([[u[0], u[1], u[2]], [0.0, u[3], u[4]], [0.0, 0.0, u[5]]])
    return np.linalg.inv(U.T @ U)


def pin_split_gaussians():
    """Half-normal split: an axis-aligned Gaussian with standard deviations (0.3, 0.1, 0.05) splits
    along x into means mu +- 0.3 sqrt(2/pi) e_x with x deviation 0.3 sqrt(1 - 2/pi); for random
    Gaussians the equal mixture of the two children has exactly the parent's mean and
    covariance; weights and colours take the given noise."""
    mu = np.array([0.1, -0.2, 0.3])
    sd = np.array([0.3, 0.1, 0.05])
    out = O.split_gaussians(mu[None], [[1 / sd[0], 0, 0, 1 / sd[1], 0, 1 / sd[2]]], [0.7])
    d = 0.3 * math.sqrt(2 / math.pi)
    _close(out["means"], [mu + [d, 0, 0], mu - [d, 0, 0]], 1e-14, 1e-14, "axis-aligned split means")
    sd2 = sd * [math.sqrt(1 - 2 / math.pi), 1, 1]
    _close(out["prec"], np.tile([1 / sd2[0], 0, 0, 1 / sd2[1], 0, 1 / sd2[2]], (2, 1)), 1e-12, 1e-12,
           "axis-aligned split precision")
    _close(out["weights"], [0.7, 0.7], 1e-15, 0.0, "split weights without noise")
    g = _rng(51)
    for _ in range(20):
        cov, packed = _cov_and_packed(g)
        m = g.standard_normal(3)
        nw, nc = g.standard_normal(2), g.standard_normal((2, 3))
        col = g.standard_normal((1, 3))
        o = O.split_gaussians(m[None], packed[None], [1.3], col, nw, nc)
        ma, mb = o["means"]
        _close(0.5 * (ma + mb), m, 1e-12, 1e-12, "mixture mean")
        c2 = _cov_of_packed(o["prec"][0])
        _close(_cov_of_packed(o["prec"][1]), c2, 1e-12, 1e-14, "children share the covariance")
        mix = c2 + 0.5 * (np.outer(ma - m, ma - m) + np.outer(mb - m, mb - m))
        _close(mix, cov, 1e-10, 1e-12, "mixture covariance")
        _close(o["weights"], 1.3 * np.exp(nw), 1e-14, 0.0, "log-weight noise")
        _close(o["colors"], col + nc, 1e-14, 0.0, "colour noise")


def pin_prune_split_masks():
    """Removal at mean - 2 std of the weights, split at mean + 1 std of lbar (hand values)."""
    w = np.array([1.0] * 9 + [0.0])          # mean 0.9, std 0.3: 0.0 <= 0.3 removed
    assert list(O.prune_mask(w)) == [False] * 9 + [True]
    x = np.array([0.0, 0.0, 0.0, 4.0])       # mean 1, std sqrt(3): 4 >= 2.73 split
    assert list(O.split_mask(x)) == [False, False, False, True]
    # zero spread: every value sits on the threshold and the non-strict tests mark it
    assert O.split_mask(np.full(5, 2.0)).all()
    assert O.prune_mask(np.full(5, 2.0)).all()


# ---------------------------------------------------------------------------------------
# Invariances
# ---------------------------------------------------------------------------------------

def pin_scale_invariance():
    """Scene and cameras scaled by k with eta scaled by k: depth scales by k; alpha, normals and
    flow are unchanged (pins the role of eta in Eq. 7)."""
    g = _rng(22)
    sc, ea, kk, view, row, col, o, v = _flow_setup(g)
    eb = _look_at(np.array([0.5, -2.5, 1.1]))
    ref = O.render(sc, o, v, view=view, w2c_a=ea[None], intr_a=kk[None], w2c_b=eb[None], intr_b=kk[None])
    s = 2.75
    sc2 = _scene(sc.means * s, sc.prec / s, sc.weights, sc.betas, sc.eta * s)
    ea2, eb2 = ea.copy(), eb.copy()
    ea2[:, 3] *= s
    eb2[:, 3] *= s
    o2, v2 = O.pixel_rays(view, row, col, ea2[None], kk[None])
    out = O.render(sc2, o2, v2, view=view, w2c_a=ea2[None], intr_a=kk[None], w2c_b=eb2[None],
                   intr_b=kk[None])
    _close(out["depth"], s * ref["depth"], 1e-9, 1e-9, "scaled depth")
    _close(out["alpha"], ref["alpha"], 1e-9, 1e-12, "scaled alpha")
    _close(out["normal"], ref["normal"], 1e-7, 1e-8, "scaled normal")
    _close(out["flow"], ref["flow"], 1e-7, 1e-8, "scaled flow")


def pin_rigid_motion():
    """Moving the world rigidly (x -> Q x + b), with the cameras moved along, leaves depth, alpha
    and flow unchanged and rotates the normals by Q."""
    g = _rng(23)
    sc, ea, kk, view, row, col, o, v = _flow_setup(g)
    eb = _look_at(np.array([0.5, -2.5, 1.1]))
    ref = O.render(sc, o, v, view=view, w2c_a=ea[None], intr_a=kk[None], w2c_b=eb[None], intr_b=kk[None])
    q = _rot(g)
    b = g.uniform(-1, 1, 3)
    means2 = sc.means @ q.T + b
    prec2 = []
    for p in sc.prec:
        u = np.array([[p[0], p[1], p[2]], [0, p[3], p[4]], [0, 0, p[5]]])
        a2 = q @ (u.T @ u) @ q.T
        u2 = np.linalg.cholesky(a2).T
        prec2.append([u2[0, 0], u2[0, 1], u2[0, 2], u2[1, 1], u2[1, 2], u2[2, 2]])
    sc2 = _scene(means2, np.array(prec2), sc.weights)

    def move(e):
        r, t = e[:, :3], e[:, 3]
        return np.concatenate([r @ q.T, (t - r @ q.T @ b)[:, None]], axis=1)

    ea2, eb2 = move(ea), move(eb)
    o2, v2 = O.pixel_rays(view, row, col, ea2[None], kk[None])
    out = O.render(sc2, o2, v2, view=view, w2c_a=ea2[None], intr_a=kk[None], w2c_b=eb2[None],
                   intr_b=kk[None])
    _close(out["depth"], ref["depth"], 1e-9, 1e-9, "moved depth")
    _close(out["alpha"], ref["alpha"], 1e-9, 1e-12, "moved alpha")
    _close(out["normal"], ref["normal"] @ q.T, 1e-7, 1e-8, "moved normal")
    _close(out["flow"], ref["flow"], 1e-7, 1e-7, "moved flow")


def pin_normals_geometry():
    """Every n_i is perpendicular to the ray at its peak, so the blended unit normal is too."""
    g = _rng(24)
    sc, _ = _random_scene(g, 8)
    o = np.array([0.2, 0.1, -3.0])
    orig, dirs = _rays_at(g, sc.means, o)
    out = O.render(sc, orig, dirs)
    assert np.max(np.abs(np.sum(out["normal"] * dirs, axis=1))) < 1e-9
    _close(np.linalg.norm(out["normal"], axis=1), 1.0, 0, 1e-12, "unit normals")


# ---------------------------------------------------------------------------------------
# Gradients
# ---------------------------------------------------------------------------------------

def _loss(sc, orig, dirs, cam, cot):
    out = O.render(sc, orig, dirs, **cam)
    s = float(cot["depth"] @ out["depth"] + cot["alpha"] @ out["alpha"])
    s += float(np.sum(cot["normal"] * out["normal"]))
    if out["flow"] is not None:
        s += float(np.sum(cot["flow"] * out["flow"]))
    if out["color"] is not None:
        s += float(np.sum(cot["color"] * out["color"]))
    return s


def pin_gradients_fd():
    """Central differences of the oracle forward (step 1e-6 max(1,|x|)) match its adjoint for
    means, packed precision factors, weights, colours and both betas, through every output."""
    g = _rng(25)
    sc, ea, kk, view, row, col, o, v = _flow_setup(g, n=4)
    view, o, v = view[:8], o[:8], v[:8]
    eb = _look_at(np.array([0.5, -2.5, 1.1]))
    cam = dict(view=view, w2c_a=ea[None], intr_a=kk[None], w2c_b=eb[None], intr_b=kk[None])
    p = len(o)
    cot = {"depth": g.standard_normal(p), "alpha": g.standard_normal(p),
           "normal": g.standard_normal((p, 3)), "flow": g.standard_normal((p, 2)),
           "color": g.standard_normal((p, 3))}
    colors = g.standard_normal((sc.n, 3))
    for eta in (1.0, 1.7):
        sc = O.OracleScene.of(sc.means, sc.prec, sc.weights, (B1 * 0.3, B2), eta, colors)
        an = O.backward(sc, o, v, cot, **cam)
        for name in ("means", "prec", "weights", "betas", "colors"):
            base = getattr(sc, name)
            fd = np.zeros_like(base)
            flat, fdf = base.reshape(-1), fd.reshape(-1)
            for j in range(flat.size):
                h = 1e-6 * max(1.0, abs(flat[j]))
                x0 = flat[j]
                flat[j] = x0 + h
                fp = _loss(sc, o, v, cam, cot)
                flat[j] = x0 - h
                fm = _loss(sc, o, v, cam, cot)
                flat[j] = x0
                fdf[j] = (fp - fm) / (2 * h)
            scale = max(1.0, float(np.max(np.abs(fd))))
            _close(an[name], fd, 1e-6, 1e-6 * scale, f"FD gradient {name} (eta={eta})")


def pin_colour_blend():
    """Colours c_i = sigmoid(q_i) blend by Eq. (3): one Gaussian renders sigmoid(q) exactly; two
    render s c_1 + (1 - s) c_2 with s = sigma(z_1 - z_2) from one-Gaussian renders; beta = 0 gives
    the plain mean of the colours."""
    g = _rng(29)
    sc, _ = _random_scene(g, 2, spread=0.3)
    q = g.standard_normal((2, 3)) * 2.0
    c = 1.0 / (1.0 + np.exp(-q))
    o = np.array([0.3, -0.2, -3.0])
    orig, dirs = _rays_at(g, np.repeat(sc.means, 3, axis=0), o, jitter=0.05)
    one = O.OracleScene.of(sc.means[[0]], sc.prec[[0]], sc.weights[[0]], sc.betas, sc.eta, q[[0]])
    _close(O.render(one, orig, dirs)["color"], np.tile(c[0], (len(orig), 1)), 1e-14, 1e-15, "one colour")
    t1, d1, _ = _single_terms(sc, 0, orig, dirs)
    t2, d2, _ = _single_terms(sc, 1, orig, dirs)
    s = 1 / (1 + np.exp(-((B1 * d1 - B2 * t1) - (B1 * d2 - B2 * t2))))
    two = O.OracleScene.of(sc.means, sc.prec, sc.weights, sc.betas, sc.eta, q)
    _close(O.render(two, orig, dirs)["color"], s[:, None] * c[0] + (1 - s)[:, None] * c[1], 1e-9, 1e-9,
           "two-colour blend")
    flat = O.OracleScene.of(sc.means, sc.prec, sc.weights, (0.0, 0.0), sc.eta, q)
    _close(O.render(flat, orig, dirs)["color"], np.tile(c.mean(axis=0), (len(orig), 1)), 1e-12, 1e-12,
           "zero-beta colour mean")


def pin_isotropic_depth_gradient():
    """One isotropic Gaussian: t_f = (mu - o).v, so d t_f / d mu = v."""
    g = _rng(26)
    mu = g.uniform(-1, 1, 3)
    o = np.array([0.0, 0.0, -3.0])
    v = _unit(mu + 0.1 * g.standard_normal(3) - o)
    sc = _scene(mu[None], _packed_iso(0.2)[None], [0.8])
    gr = O.backward(sc, o[None], v[None], {"depth": np.ones(1)})
    _close(gr["means"][0], v, 1e-10, 1e-12, "d t_f / d mu")
    _close(gr["betas"], 0.0, 0, 1e-12, "d t_f / d beta")


def pin_two_gaussian_beta_gradient():
    """N = 2: d t_f / d beta1 = (t1 - t2) s (1 - s) (d1 - d2) and
    d t_f / d beta2 = -(t1 - t2)^2 s (1 - s) / eta, s = sigma(z1 - z2)."""
    g = _rng(27)
    eta = 1.3
    sc, _ = _random_scene(g, 2, spread=0.3, eta=eta)
    o = np.array([0.3, -0.2, -3.0])
    orig, dirs = _rays_at(g, sc.means, o, jitter=0.03)
    for r in range(len(orig)):
        t1, d1, _ = _single_terms(sc, 0, orig[[r]], dirs[[r]])
        t2, d2, _ = _single_terms(sc, 1, orig[[r]], dirs[[r]])
        z1, z2 = B1 * d1[0] - B2 / eta * t1[0], B1 * d2[0] - B2 / eta * t2[0]
        s = 1 / (1 + math.exp(-(z1 - z2)))
        gr = O.backward(sc, orig[[r]], dirs[[r]], {"depth": np.ones(1)})
        _close(gr["betas"][0], (t1[0] - t2[0]) * s * (1 - s) * (d1[0] - d2[0]), 1e-8, 1e-12,
               "d t_f / d beta1")
        _close(gr["betas"][1], -((t1[0] - t2[0]) ** 2) * s * (1 - s) / eta, 1e-8, 1e-12,
               "d t_f / d beta2")


def pin_loss_gradient():
    """The loss gradient equals central differences of the loss value (away from the kinks of the
    clamp and of |x|), and a hand-computed single-ray value: alpha = 0.5, target mask 1, depth
    error 0.25 with w_depth 2, flow error (0.1, -0.2) squared L2 with w_flow 3 gives
    L = log 2 + 0.5 + 0.15."""
    L, _ = O.loss_grad([1.25], [0.5], [1.0], [1.0], flow=[[0.1, -0.2]], flow_t=[[0.0, 0.0]],
                       w_depth=2.0, w_flow=3.0, flow_norm=2)
    _close(L, math.log(2.0) + 0.5 + 0.15, 1e-14, 1e-14, "hand-computed loss")
    L, _ = O.loss_grad([1.0], [0.5], [1.0], [1.0], color=[[0.2, 0.5, 0.9]], color_t=[[0.1, 0.5, 1.0]],
                       w_color=4.5)
    _close(L, math.log(2.0) + 4.5 * 0.2, 1e-14, 1e-14, "hand-computed colour loss")
    g = _rng(28)
    p = 16
    d, dt = g.uniform(1, 4, p), g.uniform(1, 4, p)
    a, at = g.uniform(0.01, 0.99, p), g.uniform(0, 1, p)
    f, ft = g.standard_normal((p, 2)), g.standard_normal((p, 2))
    c, ct = g.uniform(0, 1, (p, 3)), g.uniform(0, 1, (p, 3))
    for norm in (1, 2):
        _, gr = O.loss_grad(d, a, dt, at, f, ft, 1.5, 2.5, norm, c, ct, 4.5)
        for name, x in (("depth", d), ("alpha", a), ("flow", f), ("color", c)):
            fd = np.zeros_like(x)
            flat = x.reshape(-1)
            for j in range(flat.size):
                h = 1e-6
                x0 = flat[j]
                flat[j] = x0 + h
                lp, _ = O.loss_grad(d, a, dt, at, f, ft, 1.5, 2.5, norm, c, ct, 4.5)
                flat[j] = x0 - h
                lm, _ = O.loss_grad(d, a, dt, at, f, ft, 1.5, 2.5, norm, c, ct, 4.5)
                flat[j] = x0
                fd.reshape(-1)[j] = (lp - lm) / (2 * h)
            _close(gr[name], fd, 1e-6, 1e-7, f"loss gradient {name} (q={norm})")
    # outside the clamp range the alpha gradient vanishes
    _, gr = O.loss_grad([1.0, 1.0], [0.0, 1.0], [1.0, 1.0], [0.5, 0.5])
    assert np.all(gr["alpha"] == 0.0)


ALL_PINS = [
    pin_isotropic_closed_form, pin_bruteforce_peak, pin_interop_alpha, pin_alpha_identities,
    pin_two_gaussian_blend, pin_zero_betas_mean, pin_permutation, pin_pixel_ray_hand_case,
    pin_rays_reproject, pin_dir_rays, pin_flow_equal_poses, pin_flow_rotation_homography, pin_flow_translation,
    pin_scale_invariance, pin_rigid_motion, pin_normals_geometry, pin_gradients_fd,
    pin_isotropic_depth_gradient, pin_two_gaussian_beta_gradient, pin_loss_gradient,
    pin_colour_blend, pin_flow_both_directions, pin_max_weight,
    pin_composite_single_gaussian, pin_composite_sorted_reference, pin_composite_ties,
    pin_composite_background, pin_composite_scale_invariance, pin_composite_gradients_fd,
    pin_split_statistic, pin_split_gaussians, pin_prune_split_masks,
]
