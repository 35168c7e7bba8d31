"""Shared pieces of the GPU parity tests: tolerances, the gradient comparison
and progress lines (a GPU test prints what it is about to run, flushed, so a
failing run names its case)."""
import sys

import numpy as np

PIX_TOL = 1e-4   # |C_gpu - C_oracle| per pixel and channel, oracle in matched mode
GRAD_TOL = 1e-3  # per tensor (relative L2) and per element, see grad_errors
FLOOR = 1e-2     # the per-element relative bar applies to at least FLOOR x the rms or the magnitude
# Relative band around the skip threshold eps_alpha and the stop threshold t_min
# inside which the kernel's float32 decision may differ from the oracle's FP64
# one (the kernel's alpha is good to ~1e-4 relative near eps_alpha and its T to
# ~1e-3 after a few opaque convexes; the band leaves a margin of 10 and more).
DECISION_TAU = 1e-2
NAMES = ("points", "delta", "sigma", "opacity", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def grad_errors(g_gpu, g_ref, scales=None):
    """{name: (relative L2 error, worst element error)} of GPU gradients (torch
    tensors or arrays) against reference arrays.

    The element error is max(|gpu - ref| - A, 0) / max(|ref|, FLOOR rms(ref), FLOOR M);
    it passes at <= GRAD_TOL, i.e. |gpu - ref| <= GRAD_TOL max(...) + A,
    where, when scales = oracle.backward_magnitude(...) is given, M is the
    element's sum of |products| (a sum that cancels is only good to a few
    float32 roundoffs of M) and A the sum over the pairs whose skip / stop
    decision is within DECISION_TAU of its threshold (either side may take
    them).  Without scales M = A = 0."""
    out = {}
    for k in NAMES:
        a = g_gpu[k]
        a = (a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)).astype(np.float64).ravel()
        b = np.asarray(g_ref[k], np.float64).ravel()
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(nb, 1e-300)
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        base = np.maximum(np.abs(b), FLOOR * rms + 1e-300)
        d = np.abs(a - b)
        if scales is not None:
            M = np.asarray(scales[0][k], np.float64).ravel()
            A = np.asarray(scales[1][k], np.float64).ravel()
            base = np.maximum(base, FLOOR * M)
            d = np.maximum(d - A, 0.0)
        elem = d / base
        out[k] = (float(rel), float(elem.max()) if b.size else 0.0)
    return out


def grad_check(g_gpu, g_ref, label, scales=None):
    worst = grad_errors(g_gpu, g_ref, scales)
    say(f"[{label}] grad rel-L2 / worst element: " + ", ".join(f"{k} {v[0]:.1e}/{v[1]:.1e}" for k, v in worst.items()))
    for k, (rel, el) in worst.items():
        assert rel <= GRAD_TOL, (label, k, rel)
        assert el <= GRAD_TOL, (label, k, el)
    return worst


def pixel_check(img, ref, label, sel=None):
    """Max |img - ref| over the image (or the flat pixel indices sel) against PIX_TOL."""
    a = img.detach().cpu().numpy() if hasattr(img, "detach") else np.asarray(img)
    a = a.reshape(-1, 3).astype(np.float64)
    if sel is not None:
        a = a[sel]
    err = float(np.abs(a - np.asarray(ref, np.float64).reshape(-1, 3)).max())
    say(f"[{label}] max |gpu - oracle| {err:.2e} over {a.shape[0]} pixels")
    assert err <= PIX_TOL, (label, err)
    return err
