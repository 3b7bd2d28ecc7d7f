"""Pins of the direction-filter and level-of-detail oracle (oracle/direction.py)."""
import math

import numpy as np

from oracle import direction as odir


def test_taps_closed_form():
    r, g = odir.gaussian_taps(1.0)
    assert r == 3
    e = np.exp(-np.arange(-3, 4) ** 2 / 2.0)
    np.testing.assert_allclose(g, e / e.sum(), rtol=1e-15)
    r, g = odir.gaussian_taps(0.5)
    assert r == 2 and abs(g.sum() - 1) < 1e-15
    # the centre weight of sigma = 1: 1 / (1 + 2 e^-1/2 + 2 e^-2 + 2 e^-9/2)
    c = 1.0 / (1 + 2 * math.exp(-0.5) + 2 * math.exp(-2) + 2 * math.exp(-4.5))
    assert abs(odir.gaussian_taps(1.0)[1][3] - c) < 1e-15


def test_filter_invariants():
    rng = np.random.default_rng(0)
    l, D = 12, 3
    const = np.broadcast_to(rng.uniform(size=D), (l, l, D))
    np.testing.assert_allclose(odir.filter_direction(const, 1.3), const, rtol=1e-14)
    b = rng.uniform(size=(l, l, D))
    assert np.array_equal(odir.filter_direction(b, 0), b)
    # rows summing to 1 still do (convex combination)
    s = b / b.sum(axis=2, keepdims=True)
    np.testing.assert_allclose(odir.filter_direction(s, 0.8).sum(axis=2), 1.0, rtol=1e-14)
    # linearity, and equivariance under a periodic shift in phi
    c = rng.uniform(size=(l, l, D))
    np.testing.assert_allclose(odir.filter_direction(2 * b - c, 0.7),
                               2 * odir.filter_direction(b, 0.7) - odir.filter_direction(c, 0.7),
                               atol=1e-13)
    np.testing.assert_allclose(odir.filter_direction(np.roll(b, 5, axis=1), 0.9),
                               np.roll(odir.filter_direction(b, 0.9), 5, axis=1), atol=1e-14)


def test_filter_impulse_and_edges():
    l = 16
    b = np.zeros((l, l, 1))
    b[8, 0, 0] = 1.0  # away from the theta edges, on the phi seam
    r, g = odir.gaussian_taps(1.0)
    out = odir.filter_direction(b, 1.0)[..., 0]
    expect = np.zeros((l, l))
    for a in range(-r, r + 1):
        for c in range(-r, r + 1):
            expect[8 + a, c % l] += g[a + r] * g[c + r]
    np.testing.assert_allclose(out, expect, atol=1e-16)
    # theta edge: rows clamp, so a table that depends on theta only keeps the
    # edge row's mass: row 0 of a step table (1 on row 0, 0 elsewhere) is
    # sum_{a <= 0} g(a) once row -a clamps to row 0
    b = np.zeros((l, l, 1))
    b[0] = 1.0
    out = odir.filter_direction(b, 1.0)
    np.testing.assert_allclose(out[0, :, 0], g[:r + 1].sum(), rtol=1e-14)
    np.testing.assert_allclose(out[1, :, 0], g[:r].sum(), rtol=1e-14)


def test_lod_select():
    K = [[100.0, 0, 50], [0, 100.0, 50], [0, 0, 1]]
    c2w = np.eye(3, 4)
    c2w[:, 3] = [0, 0, -4.0]  # 4 units from the centre of a [-1, 1]^3 box
    ks = [256, 512, 768, 128]
    # footprint = 4 / 100 = 0.04; voxel edge 2 / k <= ratio * 0.04
    assert odir.lod_select(ks, (-1,) * 3, (1,) * 3, K, c2w, 1.0) == 3      # 2/128 = 0.0156 ok
    assert odir.lod_select(ks, (-1,) * 3, (1,) * 3, K, c2w, 0.3) == 0      # 2/k <= 0.012: k >= 256
    assert odir.lod_select(ks, (-1,) * 3, (1,) * 3, K, c2w, 0.05) == 2     # none: the finest
    c2w[:, 3] = [0, 0, -40.0]
    assert odir.lod_select(ks, (-1,) * 3, (1,) * 3, K, c2w, 0.05) == 3     # far away: coarsest
