"""The tile bound the kernels use to pass over (ray tile, Gaussian) pairs (CPU only).

For a tile of unit ray directions v with unit centre direction c and largest |v - c| = rho, and a
Gaussian with Sigma^-1 = U^T U and mean mu' relative to the camera centre, the kernels bound every
ray's squared Mahalanobis distance at its density peak from below by

    m(v) >= max(0, sqrt(m(c)) - |U|_2 t_max rho)^2,   t_max = |U mu'| |U^-1|_2 >= |t(v)|,

with the 2-norms bounded by sqrt(|.|_1 |.|_inf).  This test restates that bound in FP64 and checks
it, and |t(v)| <= t_max, against the exact peak of every ray on random tiles and random
anisotropic Gaussians (scale ratios up to 100, means near and far, behind the camera too), so
that a slip in its derivation (a norm that is not an upper bound, a missing factor) fails here.
"""
from __future__ import annotations

import numpy as np


def _peak(U, mu, v):
    """Exact peak depth t and m = |U(t v - mu)|^2 of unit rays v [R,3] for one Gaussian."""
    a = v @ U.T
    b = U @ mu
    t = (a @ b) / (a * a).sum(1)
    r = (t[:, None] * v) @ U.T - b[None]
    return t, (r * r).sum(1)


def _bound(U, mu, c, rho):
    """The kernels' lower bound of m over the tile, and their bound of |t|."""
    _, mc = _peak(U, mu, c[None])
    Ui = np.linalg.inv(U)
    norm2 = lambda A: np.sqrt(np.abs(A).sum(0).max() * np.abs(A).sum(1).max())  # noqa: E731 (>= |A|_2)
    tmax = np.linalg.norm(U @ mu) * norm2(Ui)
    lo = max(0.0, np.sqrt(mc[0]) - norm2(U) * tmax * rho)
    return lo * lo, tmax


def test_tile_bound_is_a_lower_bound_of_every_rays_m():
    g = np.random.Generator(np.random.PCG64(11))
    checked = 0
    for _ in range(400):
        # a Gaussian: random rotation, log-uniform scales over two decades, upper-triangular U
        q = g.standard_normal(4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        s = np.exp(g.uniform(np.log(0.005), np.log(0.5), 3))
        U = np.linalg.cholesky(R @ np.diag(s ** -2.0) @ R.T).T
        mu = g.uniform(-1, 1, 3) + np.array([0.0, 0.0, g.choice([3.0, 0.5, -2.0])])
        # a tile: rays around a random centre within an angle of up to a few degrees
        c = g.standard_normal(3) + np.array([0.0, 0.0, 3.0])
        c /= np.linalg.norm(c)
        spread = g.uniform(0.002, 0.03)
        v = c[None] + spread * g.standard_normal((64, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        cc = v.sum(0)
        cc /= np.linalg.norm(cc)
        rho = np.linalg.norm(v - cc[None], axis=1).max()
        t, m = _peak(U, mu, v)
        lo2, tmax = _bound(U, mu, cc, rho)
        assert np.all(np.abs(t) <= tmax * (1 + 1e-12)), (np.abs(t).max(), tmax)
        assert np.all(m >= lo2 * (1 - 1e-12) - 1e-9), (m.min(), lo2)
        checked += int(lo2 > 0)
    # the bound is not vacuous: it is positive on a good share of these tiles
    assert checked > 100, checked
