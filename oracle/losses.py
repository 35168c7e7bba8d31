"""Oracle of the training step's photometric loss (paper Sec. 3.3, Eq. loss):
L = (1 - lambda) L1 + lambda (1 - SSIM), written with plain PyTorch float64 CPU
ops; its gradient comes from torch autograd.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path; it
shares no code with the HIP library.

SSIM follows the convention of 3DGS, which the paper follows for this loss:
an 11x11 Gaussian window with sigma 1.5, zero padding ("same" size), C1 =
0.01^2, C2 = 0.03^2, the map averaged over pixels and channels.  The mask term
of the equation belongs to a learnable-mask extension outside the rasterizer.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(radius: int = 5, sigma: float = 1.5) -> torch.Tensor:
    t = torch.arange(-radius, radius + 1, dtype=torch.float64)
    g = torch.exp(-t * t / (2 * sigma * sigma))
    return g / g.sum()


def _blur(img: torch.Tensor) -> torch.Tensor:
    """Same-size 2D correlation with the window's outer product, zero padding;
    img [1][3][H][W]."""
    g = window()
    w2 = torch.outer(g, g)[None, None].repeat(3, 1, 1, 1)
    return F.conv2d(img, w2, padding=5, groups=3)


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """SSIM per pixel and channel of [H][W][3] images (float64)."""
    X = x.permute(2, 0, 1)[None]
    Y = y.permute(2, 0, 1)[None]
    mx, my = _blur(X), _blur(Y)
    sxx = _blur(X * X) - mx * mx
    syy = _blur(Y * Y) - my * my
    sxy = _blur(X * Y) - mx * my
    s = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return s[0].permute(1, 2, 0)


def loss_and_grad(rgb: np.ndarray, target: np.ndarray, lam: float = 0.2):
    """(L, dL/drgb) for [H][W][3] arrays, float64."""
    x = torch.tensor(np.asarray(rgb, np.float64), requires_grad=True)
    y = torch.tensor(np.asarray(target, np.float64))
    L = (1 - lam) * (x - y).abs().mean() + lam * (1 - ssim_map(x, y).mean())
    L.backward()
    return float(L.detach()), x.grad.numpy()
