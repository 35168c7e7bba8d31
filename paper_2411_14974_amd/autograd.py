"""torch.autograd wrapper of the rasterizer: the hand-written backward kernels
produce gradients for points, delta, sigma, opacity and SH (paper Sec. 3.3's
optimised parameters).  The backward recomputes each pair's indicator per tile
from the forward state's per-pixel (last list position, transmittance); no
per-pixel-per-convex state is stored."""
from __future__ import annotations

import torch

from .binding import DeviceScene, Renderer, make_camera, make_params


class ConvexRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, delta, sigma, opacity, sh, renderer: Renderer, cam, params):
        # 16-bit parameters (the light model) are rendered from their own
        # storage; autograd casts the float32 gradients back to their dtype
        dtype = points.dtype if points.dtype in (torch.float16, torch.bfloat16) else torch.float32
        scene = DeviceScene(points.detach(), delta.detach(), sigma.detach(), opacity.detach(), sh.detach(),
                            device=points.device, dtype=dtype)
        rgb, state = renderer.forward(scene, cam, params, want_state=True)
        ctx.renderer, ctx.state = renderer, state
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        grads = ctx.renderer.backward(ctx.state, grad_rgb.float().contiguous())
        ctx.state.release()
        ctx.state = None
        return grads["points"], grads["delta"], grads["sigma"], grads["opacity"], grads["sh"], None, None, None


def render(points, delta, sigma, opacity, sh, renderer: Renderer, cam, params=None):
    """Differentiable render: returns the [H][W][3] image."""
    camS = make_camera(cam) if not hasattr(cam, "_fields_") else cam
    return ConvexRender.apply(points, delta, sigma, opacity, sh, renderer, camS, params or make_params())
