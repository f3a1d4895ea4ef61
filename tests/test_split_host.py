"""The library's host-side removal and split of Gaussians (Sec. 8) against the oracle.

These entry points run on host arrays, so the comparison runs without a GPU.
"""

from __future__ import annotations

import math

import numpy as np
import pytest

import oracle as O
import workloads as W

fmb = pytest.importorskip("paper_2308_14737_amd")
from paper_2308_14737_amd import split as SP  # noqa: E402


def _cov(u):
    U = np.array([[u[0], u[1], u[2]], [0.0, u[3], u[4]], [0.0, 0.0, u[5]]], np.float64)
    return np.linalg.inv(U.T @ U)


def test_split_gaussians_matches_oracle():
    g = np.random.Generator(np.random.PCG64(60))
    sc = W.make_scene(g, 200, g.uniform(-1, 1, (200, 3)))
    col = g.standard_normal((200, 3)).astype(np.float32)
    nw = (0.1 * g.standard_normal(400)).astype(np.float32)
    nc = (0.1 * g.standard_normal((400, 3))).astype(np.float32)
    got = SP.split_gaussians(sc.means, sc.prec, sc.weights, col, nw, nc)
    ref = O.split_gaussians(sc.means, sc.prec, sc.weights, col, nw, nc)
    for k in ("means", "prec", "weights", "colors"):
        err = np.abs(got[k] - ref[k])
        assert np.all(err <= 2e-6 * np.abs(ref[k]) + 2e-6), (k, float(err.max()))


def test_split_isotropic_is_valid():
    """A Gaussian with a repeated dominant axis has no unique v_1: any split along that plane is
    correct, so check what is unique (mixture mean and covariance, shared child covariance)."""
    s = 0.2
    prec = np.array([[1 / s, 0, 0, 1 / s, 0, 1 / s], [1 / 0.3, 0, 0, 1 / 0.3, 0, 1 / 0.1]], np.float32)
    means = np.array([[0.0, 0.1, 0.2], [0.3, 0.0, -0.1]], np.float32)
    got = SP.split_gaussians(means, prec, np.ones(2, np.float32))
    for i in range(2):
        ma, mb = got["means"][2 * i].astype(np.float64), got["means"][2 * i + 1].astype(np.float64)
        c = _cov(got["prec"][2 * i])
        assert np.allclose(_cov(got["prec"][2 * i + 1]), c, rtol=1e-6, atol=1e-9)
        assert np.allclose(0.5 * (ma + mb), means[i], atol=1e-6)
        mix = c + 0.5 * (np.outer(ma - means[i], ma - means[i]) + np.outer(mb - means[i], mb - means[i]))
        assert np.allclose(mix, _cov(prec[i]), rtol=1e-5, atol=1e-8)
        shift = np.linalg.norm(ma - means[i])
        assert abs(shift - math.sqrt(np.linalg.eigvalsh(_cov(prec[i]))[-1] * 2 / math.pi)) < 1e-6


def test_masks_match_oracle():
    g = np.random.Generator(np.random.PCG64(61))
    for _ in range(5):
        w = g.uniform(0.0, 1.0, 300).astype(np.float32)
        lbar = g.exponential(1.0, 300).astype(np.float32)
        assert np.array_equal(SP.prune_mask(w), O.prune_mask(w))
        assert np.array_equal(SP.split_mask(lbar), O.split_mask(lbar))


def test_apply_split_counts():
    g = np.random.Generator(np.random.PCG64(62))
    sc = W.make_scene(g, 50, g.uniform(-1, 1, (50, 3)))
    remove = np.zeros(50, bool)
    split = np.zeros(50, bool)
    remove[[1, 2]] = True
    split[[2, 3, 4]] = True
    out = SP.apply_split(sc.means, sc.prec, sc.weights, remove=remove, split=split, rng=np.random.default_rng(1))
    assert out["means"].shape == (50 - 2 - 2 + 2 * 2, 3)
    assert out["colors"] is None
