"""Oracle of the initial convex set (paper Sec. 3.3 "Initialization and
losses"; Supp. Initialization & Hyperparameters): per cloud point, K points on
a sphere of radius radius_scale x the mean distance to its three nearest other
cloud points, at Fibonacci-sphere directions.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path; it
shares no code with the HIP library.  Nearest neighbours come from
scipy.spatial.cKDTree (a library reduction); the directions from the
Fibonacci lattice on the sphere (heights equally spaced at the cell centres,
azimuth advancing by the golden angle), in float64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

Y00 = 0.5 / math.sqrt(math.pi)


def fibonacci_directions(k: int) -> np.ndarray:
    j = np.arange(k, dtype=np.float64)
    y = 1.0 - (2.0 * j + 1.0) / k
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1.0 - y * y)
    return np.stack([np.cos(phi) * r, y, np.sin(phi) * r], axis=1)


def mean_knn3(xyz: np.ndarray) -> np.ndarray:
    """Mean distance to the (up to) three nearest other points."""
    p = np.asarray(xyz, np.float64)
    n = p.shape[0]
    if n <= 1:
        return np.zeros(n)
    kq = min(4, n)
    d, _ = cKDTree(p).query(p, k=kq)
    return d[:, 1:].mean(axis=1)


def init_from_points(xyz, rgb, k, sh_degree, radius_scale=1.2, radius_min=1e-7, delta0=0.1, sigma0=0.00095,
                     opacity0=0.1):
    p = np.asarray(xyz, np.float64)
    n = p.shape[0]
    r = radius_scale * np.maximum(mean_knn3(p), radius_min)
    pts = p[:, None, :] + r[:, None, None] * fibonacci_directions(k)[None]
    nc = (sh_degree + 1) ** 2
    sh = np.zeros((n, nc, 3))
    if rgb is not None:
        sh[:, 0, :] = (np.asarray(rgb, np.float64) - 0.5) / Y00
    return pts, np.full(n, delta0), np.full(n, sigma0), np.full(n, opacity0), sh, r
