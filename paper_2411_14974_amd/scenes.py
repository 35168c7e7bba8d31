"""Seeded synthetic scenes and cameras shaped like the paper's workloads.

This module only draws inputs: it holds none of the renderer's arithmetic, and
both the HIP path and the CPU oracle read the arrays it returns.  Every draw
uses numpy's PCG64 ``default_rng`` with the seed ``1000 * config + variant``,
in the order written in each function.

The paper fits real scenes (Tanks&Temples, Deep Blending, Mip-NeRF360; its
Sec. 4 "Datasets") that are not available here; these scenes stand in for them
at the paper's scale: its memory column of Table 1 divided by 69 FP32
parameters per convex (Sec. 4 "Implementation details") gives about 1 to 2.4
million convexes per scene.

Scene arrays are float32:
    points  [N][K][3]   world space
    delta   [N]         smoothness  (> 0, activated)
    sigma   [N]         sharpness   (> 0, activated)
    opacity [N]         in [0, 1]   (activated)
    sh      [N][(D+1)^2][3]
The light model (paper Sec. 4.2) stores the same parameters in 16-bit
precision; ``Scene.stored`` gives the float32 values such a scene holds
(round to nearest even), which the oracle and a float32 render read.
Camera: pinhole, world->camera rotation R (rows = camera x right, y down,
z forward) and translation t, focal lengths and principal point in pixels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RESOLUTIONS_C4 = ((960, 540), (1297, 840), (1920, 1080))
RESOLUTIONS_C5 = ((256, 256), (960, 540), (1920, 1080))
SERVE_SCENE_SIZES = (200_000, 500_000, 1_000_000, 2_000_000)


@dataclass
class Scene:
    points: np.ndarray
    delta: np.ndarray
    sigma: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def k(self) -> int:
        return int(self.points.shape[1])

    @property
    def deg(self) -> int:
        return int(round(math.sqrt(self.sh.shape[1]))) - 1

    def subset(self, idx) -> "Scene":
        return Scene(*(np.ascontiguousarray(a[idx]) for a in
                       (self.points, self.delta, self.sigma, self.opacity, self.sh)))

    def stored(self, fmt: str) -> "Scene":
        """The scene as a 16-bit storage format holds it ('f16' or 'bf16'),
        as float32 arrays; 'f32' returns the scene itself."""
        if fmt == "f32":
            return self
        return Scene(*(round_to(a, fmt) for a in (self.points, self.delta, self.sigma, self.opacity, self.sh)))


def round_to(a, fmt: str) -> np.ndarray:
    """float32 values of `a` rounded to nearest, ties to even, in a 16-bit
    storage format: 'f16' (IEEE binary16) or 'bf16' (bfloat16, the upper half
    of a binary32).  Finite inputs within the format's range."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    if fmt == "f16":
        return a.astype(np.float16).astype(np.float32)
    if fmt == "bf16":
        u = a.view(np.uint32).astype(np.uint64)
        r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
        return r.astype(np.uint32).view(np.float32)
    raise ValueError(f"unknown storage format {fmt!r}")


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.float32))
    znear: float = 0.1

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        # float32 round trip so both sides read identical values
        for name in ("fx", "fy", "cx", "cy", "znear"):
            setattr(self, name, float(np.float32(getattr(self, name))))


def convexes_around(rng: np.random.Generator, centres: np.ndarray, k: int, deg: int) -> Scene:
    """K points on a sphere of random radius around each centre, plus appearance.

    Draw order: radius, directions, delta, sigma, opacity, SH."""
    n = centres.shape[0]
    s = np.exp(rng.normal(math.log(0.05), 0.5, n))
    u = rng.normal(size=(n, k, 3))
    u /= np.linalg.norm(u, axis=2, keepdims=True)
    points = centres[:, None, :] + s[:, None, None] * u
    delta = np.exp(rng.uniform(0.0, math.log(50.0), n))
    sigma = np.exp(rng.uniform(0.0, math.log(20.0), n))
    opacity = rng.uniform(0.1, 0.9, n)
    if deg == 0:
        # with the degree-0 basis constant 1/(2 sqrt(pi)) this range spans colours [0, 1]
        sh = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), (n, 1, 3))
    else:
        sh = rng.normal(0.0, 0.2, (n, (deg + 1) ** 2, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(points), f32(delta), f32(sigma), f32(opacity), f32(sh))


def uniform_centres(rng, n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)):
    return np.stack([rng.uniform(lo[i], hi[i], n) for i in range(3)], axis=1)


def gmm_centres(rng, n, components=64):
    """64-component isotropic mixture: means U[-1,1]^3, std U[0.1,0.5], equal weights."""
    means = rng.uniform(-1.0, 1.0, (components, 3))
    stds = rng.uniform(0.1, 0.5, components)
    comp = rng.integers(0, components, n)
    return means[comp] + stds[comp, None] * rng.normal(size=(n, 3))


def orbit_camera(rng, width, height, radius=4.0) -> Camera:
    """Random pose on a sphere of the given radius looking at the origin, fx = fy = W."""
    while True:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        if abs(v[1]) <= 0.99:
            break
    campos = radius * v
    f = -v
    r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    R = np.stack([r, dn, f])
    t = -R @ campos
    return Camera(width, height, float(width), float(width), width / 2.0, height / 2.0, R, t)


def origin_camera(width=128, height=128, focal=128.0) -> Camera:
    return Camera(width, height, focal, focal, width / 2.0, height / 2.0)


# ------------------------------------------------------------------ configs --

def config1(variant: int = 0, n: int = 1000):
    """1k convexes, K=6, SH degree 0, camera at the origin looking +z, 128x128."""
    rng = np.random.default_rng(1000 * 1 + variant)
    centres = uniform_centres(rng, n, (-1.0, -1.0, 2.0), (1.0, 1.0, 6.0))
    return convexes_around(rng, centres, 6, 0), origin_camera()


def config2(variant: int = 0, n: int = 100_000, width: int = 1297, height: int = 840, k: int = 6, deg: int = 3):
    """100k convexes, K=6, SH degree 3, centres U[-1,1]^3, one orbit pose, L1 target."""
    rng = np.random.default_rng(1000 * 2 + variant)
    centres = uniform_centres(rng, n)
    scene = convexes_around(rng, centres, k, deg)
    cam = orbit_camera(rng, width, height)
    target = rng.uniform(0.0, 1.0, (height, width, 3)).astype(np.float32)
    return scene, cam, target


def config3(variant: int = 0, n: int = 1_000_000, width: int = 1920, height: int = 1080, k: int = 6, deg: int = 3):
    """1M convexes from a 64-component mixture (uneven tile loads), 1920x1080, L1 target."""
    rng = np.random.default_rng(1000 * 3 + variant)
    centres = gmm_centres(rng, n)
    scene = convexes_around(rng, centres, k, deg)
    cam = orbit_camera(rng, width, height)
    target = rng.uniform(0.0, 1.0, (height, width, 3)).astype(np.float32)
    return scene, cam, target


def config4(variant: int = 0, n: int = 500_000, views: int = 32, resolutions=RESOLUTIONS_C4):
    """The mixture scene with 500k convexes seen from 32 orbit poses of mixed size."""
    rng = np.random.default_rng(1000 * 4 + variant)
    centres = gmm_centres(rng, n)
    scene = convexes_around(rng, centres, 6, 3)
    picks = rng.integers(0, len(resolutions), views)
    cams = [orbit_camera(rng, *resolutions[p]) for p in picks]
    targets = [rng.uniform(0.0, 1.0, (c.height, c.width, 3)).astype(np.float32) for c in cams]
    return scene, cams, targets


def serve_scene(index: int, sizes=SERVE_SCENE_SIZES) -> Scene:
    """Resident scene ``index`` of the serving workload (mixture generator)."""
    rng = np.random.default_rng(1000 * 5 + index)
    centres = gmm_centres(rng, sizes[index])
    return convexes_around(rng, centres, 6, 3)


def serve_requests(rate: float, duration_s: float, n_scenes: int = 4, variant: int = 0,
                   resolutions=RESOLUTIONS_C5):
    """Poisson arrivals: list of (arrival_s, scene_id, Camera)."""
    rng = np.random.default_rng(1000 * 5 + 100 + variant)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            return out
        sid = int(rng.integers(0, n_scenes))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append((t, sid, orbit_camera(rng, w, h)))
