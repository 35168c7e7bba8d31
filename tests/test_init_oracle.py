"""Pins of the initialisation oracle: the Fibonacci directions (unit vectors,
equally spaced heights, golden-angle azimuth steps, balanced), the 3-NN mean
against brute force, and the SH colour round trip."""
import math

import numpy as np

from oracle import init as I


def test_fibonacci_directions():
    for k in (3, 6, 8, 100):
        d = I.fibonacci_directions(k)
        np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
        np.testing.assert_allclose(np.diff(d[:, 1]), -2.0 / k, atol=1e-15)        # equally spaced heights
        assert abs(d[:, 1].sum()) < 1e-12                                          # symmetric about the equator
        az = np.arctan2(d[:, 2], d[:, 0])
        step = np.mod(np.diff(az), 2 * math.pi)
        np.testing.assert_allclose(step, math.pi * (3 - math.sqrt(5)), atol=1e-12)
    # many points: nearly uniform, the centroid tends to the centre
    assert np.linalg.norm(I.fibonacci_directions(2000).mean(axis=0)) < 1e-3


def test_knn3_mean_against_brute_force():
    rng = np.random.default_rng(0)
    p = rng.normal(size=(300, 3))
    d = np.linalg.norm(p[:, None] - p[None], axis=2)
    np.fill_diagonal(d, np.inf)
    want = np.sort(d, axis=1)[:, :3].mean(axis=1)
    np.testing.assert_allclose(I.mean_knn3(p), want, rtol=1e-12)
    # two points: the one other point
    np.testing.assert_allclose(I.mean_knn3(np.array([[0, 0, 0], [0, 3, 4.0]])), [5.0, 5.0])


def test_initial_convex_geometry_and_colour():
    rng = np.random.default_rng(1)
    xyz = rng.uniform(-1, 1, (200, 3))
    rgb = rng.uniform(0, 1, (200, 3))
    pts, dl, sg, op, sh, r = I.init_from_points(xyz, rgb, 6, 3)
    np.testing.assert_allclose(pts.mean(axis=1)[:, 1], xyz[:, 1], atol=1e-12)   # heights balance out
    np.testing.assert_allclose(np.linalg.norm(pts - xyz[:, None], axis=2), r[:, None].repeat(6, 1), rtol=1e-12)
    np.testing.assert_allclose(0.5 + I.Y00 * sh[:, 0], rgb, atol=1e-12)          # colour reproduced
    assert np.all(sh[:, 1:] == 0) and np.all(dl == 0.1) and np.all(op == 0.1)
