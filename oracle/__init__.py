"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  It shares no code with
the HIP library; only the seeded input generator feeds both.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAXK = 8

MODE_EXACT = 0
MODE_MATCHED = 1
EPS_ALPHA = 1e-6
T_MIN = 1e-5
DEGENERATE = 256  # or-ed into Convex.status: a near-collinear point triple makes the hull ill-posed


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP contraction off so the float32 key is pinned)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32), ("deg", C.c_int32), ("pad", C.c_int32),
                ("points", C.c_void_p), ("delta", C.c_void_p), ("sigma", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class Convex(C.Structure):
    _fields_ = [("status", C.c_int32), ("T", C.c_int32), ("hull", C.c_int32 * MAXK),
                ("key", C.c_uint32), ("clampmask", C.c_int32),
                ("X", (C.c_double * 3) * MAXK), ("q", (C.c_double * 2) * MAXK),
                ("nx", C.c_double * MAXK), ("ny", C.c_double * MAXK), ("off", C.c_double * MAXK),
                ("d", C.c_double), ("dp", C.c_double), ("sp", C.c_double),
                ("rgb", C.c_double * 3), ("dir", C.c_double * 3), ("camdist", C.c_double),
                ("rect", C.c_double * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.orc_preprocess.argtypes = [vp, vp, dbl, vp]
        L.orc_render.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        L.orc_backward.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_backward_magnitude.argtypes = [vp, vp, vp, i32, vp, vp, dbl] + [vp] * 10
        L.orc_tile_candidates.argtypes = [vp, vp, dbl, i32, i32, i32, vp, i32]
        L.orc_sh_basis.argtypes = [i32, vp, vp, vp]
        L.orc_order.argtypes = [i32, vp, vp]
        L.orc_sh_basis.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _Bound:
    """FP64 copies of a scene, kept alive while the C struct points at them."""

    def __init__(self, scene):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.points, self.delta, self.sigma = f64(scene.points), f64(scene.delta), f64(scene.sigma)
        self.opacity, self.sh = f64(scene.opacity), f64(scene.sh)
        n, k = self.points.shape[:2]
        deg = int(round(np.sqrt(self.sh.shape[1]))) - 1
        self.s = _Scene(n, k, deg, 0, _ptr(self.points).value, _ptr(self.delta).value, _ptr(self.sigma).value,
                        _ptr(self.opacity).value, _ptr(self.sh).value)


def cam_array(cam) -> np.ndarray:
    return np.array([cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, *np.asarray(cam.R, np.float64).ravel(),
                     *np.asarray(cam.t, np.float64).ravel(), cam.znear], dtype=np.float64)


def par_array(mode=MODE_MATCHED, eps_alpha=EPS_ALPHA, t_min=T_MIN, bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    return np.array([eps_alpha, t_min, *bg, mode], dtype=np.float64)


def preprocess(scene, cam, rect_alpha=EPS_ALPHA):
    b = _Bound(scene)
    out = (Convex * max(scene.points.shape[0], 1))()
    camv = cam_array(cam)
    rc = lib().orc_preprocess(C.byref(b.s), _ptr(camv), rect_alpha, out)
    assert rc == 0
    return out


def order(convexes, n):
    o = np.zeros(max(n, 1), dtype=np.int32)
    m = lib().orc_order(n, convexes, _ptr(o))
    return o[:m]


def _pix(pixels):
    if pixels is None:
        return None, None
    p = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    return p, _ptr(p)


def render(scene, cam, mode=MODE_MATCHED, pixels=None, eps_alpha=EPS_ALPHA, t_min=T_MIN, bg=(0.0, 0.0, 0.0)):
    """Returns (rgb, T, ncontrib).  Whole image -> shapes [H][W][3], [H][W];
    otherwise one row per requested (u, v) pixel."""
    b = _Bound(scene)
    camv, parv = cam_array(cam), par_array(mode, eps_alpha, t_min, bg)
    p, pp = _pix(pixels)
    npix = cam.width * cam.height if p is None else p.shape[0]
    rgb = np.zeros((npix, 3), np.float64)
    T = np.zeros(npix, np.float64)
    nc = np.zeros(npix, np.int32)
    rc = lib().orc_render(C.byref(b.s), _ptr(camv), _ptr(parv), npix, pp, _ptr(rgb), _ptr(T), _ptr(nc))
    assert rc == 0
    if p is None:
        return rgb.reshape(cam.height, cam.width, 3), T.reshape(cam.height, cam.width), nc.reshape(cam.height,
                                                                                                    cam.width)
    return rgb, T, nc


def backward(scene, cam, dl_drgb, mode=MODE_MATCHED, pixels=None, eps_alpha=EPS_ALPHA, t_min=T_MIN,
             bg=(0.0, 0.0, 0.0)):
    """Gradient of sum(dl_drgb * C) w.r.t. (points, delta, sigma, opacity, sh), FP64."""
    b, camv, parv, npix, pp, g = _backward_args(scene, cam, dl_drgb, mode, pixels, eps_alpha, t_min, bg)
    out = _grad_arrays(b)
    rc = lib().orc_backward(C.byref(b.s), _ptr(camv), _ptr(parv), npix, pp, _ptr(g),
                            *(_ptr(out[k]) for k in GRAD_NAMES))
    assert rc == 0
    return out


def backward_magnitude(scene, cam, dl_drgb, mode=MODE_MATCHED, pixels=None, eps_alpha=EPS_ALPHA, t_min=T_MIN,
                       bg=(0.0, 0.0, 0.0), tau=1e-3):
    """(magnitude, ambiguous): per gradient element, the sum of |product| over
    everything the chain rule adds into it, and the same sum over the pairs
    whose matched-mode skip/stop decision lies within relative tau of its
    threshold.  Scales for judging another evaluation of backward()."""
    b, camv, parv, npix, pp, g = _backward_args(scene, cam, dl_drgb, mode, pixels, eps_alpha, t_min, bg)
    m, a = _grad_arrays(b), _grad_arrays(b)
    rc = lib().orc_backward_magnitude(C.byref(b.s), _ptr(camv), _ptr(parv), npix, pp, _ptr(g), tau,
                                      *(_ptr(m[k]) for k in GRAD_NAMES), *(_ptr(a[k]) for k in GRAD_NAMES))
    assert rc == 0
    return m, a


GRAD_NAMES = ("points", "delta", "sigma", "opacity", "sh")


def _grad_arrays(b):
    return {"points": np.zeros_like(b.points), "delta": np.zeros_like(b.delta), "sigma": np.zeros_like(b.sigma),
            "opacity": np.zeros_like(b.opacity), "sh": np.zeros_like(b.sh)}


def _backward_args(scene, cam, dl_drgb, mode, pixels, eps_alpha, t_min, bg):
    b = _Bound(scene)
    camv, parv = cam_array(cam), par_array(mode, eps_alpha, t_min, bg)
    p, pp = _pix(pixels)
    npix = cam.width * cam.height if p is None else p.shape[0]
    g = np.ascontiguousarray(dl_drgb, dtype=np.float64).reshape(npix, 3)
    return b, camv, parv, npix, pp, g


def tile_candidates(scene, cam, tile, tx, ty, eps_alpha=EPS_ALPHA):
    b = _Bound(scene)
    camv = cam_array(cam)
    cap = max(scene.points.shape[0], 1)
    ids = np.zeros(cap, np.int32)
    m = lib().orc_tile_candidates(C.byref(b.s), _ptr(camv), eps_alpha, tile, tx, ty, _ptr(ids), cap)
    assert m >= 0
    return ids[:m]


def sh_basis(deg, direction):
    d = np.ascontiguousarray(direction, dtype=np.float64)
    Y = np.zeros(16)
    dY = np.zeros(48)
    lib().orc_sh_basis(deg, _ptr(d), _ptr(Y), _ptr(dY))
    nc = (deg + 1) ** 2
    return Y[:nc], dY.reshape(16, 3)[:nc]
