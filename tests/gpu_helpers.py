"""Shared pieces of the GPU parity tests: tolerances, the gradient comparison
and progress lines (a GPU test prints what it is about to run, flushed, so a
failing run names its case)."""
import sys

import numpy as np

PIX_TOL = 1e-4   # |C_gpu - C_oracle| per pixel and channel, oracle in matched mode
GRAD_TOL = 1e-3  # per tensor (relative L2) and per element (floor 1e-2 rms of the reference)
NAMES = ("points", "delta", "sigma", "opacity", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def grad_errors(g_gpu, g_ref):
    """{name: (relative L2 error, worst element error)} of GPU gradients (torch
    tensors or arrays) against reference arrays."""
    out = {}
    for k in NAMES:
        a = g_gpu[k]
        a = (a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)).astype(np.float64).ravel()
        b = np.asarray(g_ref[k], np.float64).ravel()
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(nb, 1e-300)
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        elem = np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-300)
        out[k] = (float(rel), float(elem.max()) if b.size else 0.0)
    return out


def grad_check(g_gpu, g_ref, label):
    worst = grad_errors(g_gpu, g_ref)
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
