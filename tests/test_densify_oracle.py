"""Pins of the density-control oracle (split / prune, paper Sec. 3.3 "Adaptive
convex shape refinement"; Supp. Initialization & Hyperparameters) to facts
that hold independently of its code: closed-form radii, the children's
centres (the parent's points), scaled point differences, counts and order."""
import math

import numpy as np

from oracle import densify as D
from paper_2411_14974_amd import scenes

PAR = dict(opacity_min=0.03, size_max=1.0, split_threshold=4e-6, child_scale=0.7, child_sigma_scale=1.5,
           child_opacity_scale=0.5)


def scene_of(points, opacity=None, deg=1):
    points = np.asarray(points, np.float32)
    n = points.shape[0]
    rng = np.random.default_rng(n)
    return scenes.Scene(points, rng.uniform(1, 5, n).astype(np.float32), rng.uniform(1, 5, n).astype(np.float32),
                        np.full(n, 0.5, np.float32) if opacity is None else np.asarray(opacity, np.float32),
                        rng.normal(size=(n, (deg + 1) ** 2, 3)).astype(np.float32))


def octahedron(centre, r):
    e = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
    return np.asarray(centre, np.float64) + r * e


def test_radius_closed_form_decides_pruning():
    # octahedra of radius r (every vertex at distance r from the centre)
    radii = [0.25, 0.5, 0.99, 1.01, 2.0]
    s = scene_of([octahedron((0.3 * i, -0.2, 0.1), r) for i, r in enumerate(radii)])
    _, r2 = D._centre_radius_f32(s.points)
    np.testing.assert_allclose(np.sqrt(r2), radii, rtol=1e-6)
    code = D.classify(s, np.zeros(5), np.zeros(5), **{k: PAR[k] for k in ("opacity_min", "size_max",
                                                                           "split_threshold")})
    assert list(code) == [D.KEEP, D.KEEP, D.KEEP, D.PRUNE, D.PRUNE]


def test_opacity_threshold_and_split_statistic():
    pts = [octahedron((i, 0, 0), 0.1) for i in range(6)]
    s = scene_of(pts, opacity=[0.02, 0.03, 0.5, 0.5, 0.5, 0.01])
    accum = np.array([1.0, 0.0, 3e-6, 9e-6, 1.0, 1.0], np.float32)
    denom = np.array([1, 1, 1, 2, 0, 1], np.float32)   # means: -, 0, 3e-6, 4.5e-6, (none), -
    code = D.classify(s, accum, denom, 0.03, 1.0, 4e-6)
    # opacity < 0.03 prunes (0.03 itself stays); mean above 4e-6 splits; no views: no split;
    # prunable and splittable: pruned
    assert list(code) == [D.PRUNE, D.KEEP, D.KEEP, D.SPLIT, D.KEEP, D.PRUNE]


def test_children_are_scaled_copies_centred_at_the_parent_points():
    rng = np.random.default_rng(7)
    s = scenes.convexes_around(rng, scenes.uniform_centres(rng, 40), 6, 2)
    accum = np.where(np.arange(40) % 3 == 0, 1.0, 0.0).astype(np.float32)
    denom = np.ones(40, np.float32)
    out = D.densify(s, accum, denom, 0.0, 10.0, 0.5, 0.6, 2.0, 0.25)
    pts, dl, sg, op, sh, src = out
    nsplit = int((accum > 0.5).sum())
    assert pts.shape[0] == (40 - nsplit) + 6 * nsplit
    kept = np.nonzero(accum <= 0.5)[0]
    assert np.array_equal(src[:kept.size], kept)                         # survivors first, in order
    np.testing.assert_array_equal(pts[:kept.size], s.points[kept].astype(np.float64))
    P = s.points.astype(np.float64)
    for t, i in enumerate(np.nonzero(accum > 0.5)[0]):
        kids = pts[kept.size + 6 * t: kept.size + 6 * (t + 1)]
        assert np.all(src[kept.size + 6 * t: kept.size + 6 * (t + 1)] == i)
        # centre of child k = parent point k
        np.testing.assert_allclose(kids.mean(axis=1), P[i], atol=1e-12)
        # every child is the parent scaled by 0.6: pairwise point differences scale by 0.6
        for kd in kids:
            np.testing.assert_allclose(kd[:, None, :] - kd[None, :, :], 0.6 * (P[i][:, None, :] - P[i][None, :, :]),
                                       atol=1e-12)
        rows = slice(kept.size + 6 * t, kept.size + 6 * (t + 1))
        assert np.all(dl[rows] == s.delta[i])                            # delta kept
        np.testing.assert_allclose(sg[rows], 2.0 * s.sigma[i], rtol=1e-15)
        np.testing.assert_allclose(op[rows], 0.25 * s.opacity[i], rtol=1e-15)
        assert np.all(sh[rows] == s.sh[i])


def test_identity_when_nothing_passes():
    rng = np.random.default_rng(8)
    s = scenes.convexes_around(rng, scenes.uniform_centres(rng, 25), 5, 0)
    pts, dl, sg, op, sh, src = D.densify(s, np.zeros(25), np.ones(25), 0.0, math.inf, math.inf, 0.7, 1.5, 0.5)
    assert np.array_equal(src, np.arange(25))
    np.testing.assert_array_equal(pts, s.points.astype(np.float64))
    np.testing.assert_array_equal(sh, s.sh)


def test_decisions_agree_with_float64_wherever_rounding_cannot_decide():
    """The oracle decides in float32 in the kernel's operation order; this pin
    shares neither.  Decisions are recomputed in float64 from the definitions
    (radius about the point mean, opacity, mean statistic) on random scenes
    with thresholds placed inside the value distributions, and must agree on
    every convex whose values sit farther from a threshold than float32
    rounding can move them (relative 1e-5)."""
    rng = np.random.default_rng(4711)
    n = 20000
    s = scenes.convexes_around(rng, scenes.uniform_centres(rng, n), 6, 0)
    s.opacity[:] = rng.uniform(0.0, 0.1, n).astype(np.float32)
    accum = rng.uniform(0, 2e-5, n).astype(np.float32)
    denom = rng.integers(0, 4, n).astype(np.float32)
    P = s.points.astype(np.float64)
    r64 = np.linalg.norm(P - P.mean(axis=1, keepdims=True), axis=2).max(axis=1)
    o64 = s.opacity.astype(np.float64)
    size_max = float(np.median(r64))
    opacity_min, thr = 0.03, 4e-6
    with np.errstate(divide="ignore", invalid="ignore"):
        mean64 = np.where(denom > 0, accum.astype(np.float64) / np.maximum(denom, 1), 0.0)
    prune64 = (o64 < opacity_min) | (r64 > size_max)
    split64 = (denom > 0) & (mean64 > thr)
    want = np.where(prune64, D.PRUNE, np.where(split64, D.SPLIT, D.KEEP))
    got = D.classify(s, accum, denom, opacity_min, size_max, thr)
    rel = 1e-5
    clear = (np.abs(o64 - opacity_min) > rel * opacity_min) & (np.abs(r64 - size_max) > rel * size_max) & \
        ((denom == 0) | (np.abs(mean64 - thr) > rel * thr))
    assert clear.sum() > 0.99 * n
    assert np.array_equal(got[clear], want[clear]), np.nonzero(got[clear] != want[clear])[0][:10]
    # every outcome occurs, so each comparison is exercised
    assert all((want == c).sum() > 1000 for c in (D.PRUNE, D.KEEP, D.SPLIT))
