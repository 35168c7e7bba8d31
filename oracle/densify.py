"""Oracle of the adaptive density control step (split and prune).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path; it
shares no code with the HIP library.

Paper, Sec. 3.3 "Adaptive convex shape refinement" and Supp. "Initialization &
Hyperparameters": a convex whose sharpness-gradient statistic passes a
threshold is replaced by K convexes, one centred at each of its points, each a
scaled-down copy of it with a higher sigma and a lower opacity and the same
delta; convexes below an opacity threshold or above a size limit are removed.
The paper leaves open (readings, shared with the library's documentation):
  - the statistic: the mean over rendered views of |dL/dsigma| since the last
    step (accum / denom), split when it exceeds the threshold;
  - "size": the radius max_k |p_k - c| about the point mean c;
  - the factors for the children's sigma and opacity (caller's parameters);
  - the order: kept convexes in input order, then each split convex's K
    children in input order, child k centred at point k;
  - a convex both prunable and splittable is pruned.
The keep / split / prune decisions are taken in float32 with the kernel's
fixed operation order (a decision decided by floating point must be taken in
one precision on both sides); the children's geometry is computed in float64.
"""
from __future__ import annotations

import numpy as np

PRUNE, KEEP, SPLIT = 0, 1, 2


def _centre_radius_f32(points: np.ndarray):
    """Point mean (sums in point order, one division by K) and squared radius
    ((dx dx + dy dy) + dz dz, maximum over points), all in float32."""
    p = np.asarray(points, np.float32)
    K = p.shape[1]
    c = p[:, 0, :].copy()
    for k in range(1, K):
        c = c + p[:, k, :]
    c = c / np.float32(K)
    r2 = np.zeros(p.shape[0], np.float32)
    for k in range(K):
        d = p[:, k, :] - c
        r2 = np.maximum(r2, (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    return c, r2


def classify(scene, accum, denom, opacity_min, size_max, split_threshold):
    """PRUNE / KEEP / SPLIT per convex."""
    _, r2 = _centre_radius_f32(scene.points)
    o = np.asarray(scene.opacity, np.float32)
    a = np.asarray(accum, np.float32)
    d = np.asarray(denom, np.float32)
    smax = np.float32(size_max)
    prune = (o < np.float32(opacity_min)) | (r2 > smax * smax)
    with np.errstate(divide="ignore", invalid="ignore"):
        split = (d > 0) & (a / np.where(d > 0, d, np.float32(1)) > np.float32(split_threshold))
    return np.where(prune, PRUNE, np.where(split, SPLIT, KEEP)).astype(np.int8)


def densify(scene, accum, denom, opacity_min, size_max, split_threshold, child_scale, child_sigma_scale,
            child_opacity_scale):
    """Returns (points, delta, sigma, opacity, sh, src) of the new convex set,
    the geometry in float64."""
    code = classify(scene, accum, denom, opacity_min, size_max, split_threshold)
    P = np.asarray(scene.points, np.float64)
    K = P.shape[1]
    keep = np.nonzero(code == KEEP)[0]
    split = np.nonzero(code == SPLIT)[0]
    pts, dl, sg, op, sh, src = [P[keep]], [scene.delta[keep]], [scene.sigma[keep]], [scene.opacity[keep]], \
        [scene.sh[keep]], [keep]
    if split.size:
        c = P[split].mean(axis=1)                                       # [S][3]
        rel = P[split] - c[:, None, :]                                  # p_j - c
        # child k of convex i: p_k + s (p_j - c), j = 0..K-1
        kids = P[split][:, :, None, :] + np.float64(child_scale) * rel[:, None, :, :]   # [S][k][j][3]
        pts.append(kids.reshape(-1, K, 3))
        rep = np.repeat(split, K)
        dl.append(scene.delta[rep])
        sg.append(np.asarray(scene.sigma, np.float64)[rep] * np.float64(np.float32(child_sigma_scale)))
        op.append(np.asarray(scene.opacity, np.float64)[rep] * np.float64(np.float32(child_opacity_scale)))
        sh.append(scene.sh[rep])
        src.append(rep)
    return (np.concatenate(pts), np.concatenate(dl).astype(np.float64), np.concatenate(sg).astype(np.float64),
            np.concatenate(op).astype(np.float64), np.concatenate(sh), np.concatenate(src).astype(np.int64))
