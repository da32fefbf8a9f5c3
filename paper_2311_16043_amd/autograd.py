"""torch.autograd.Function over the visibility tracer and its adjoint.

Forward builds the BVH from the current geometry and traces every ray; backward
calls the hand-written adjoint kernel, which traces each ray again (no hit
lists are kept) and scatters d/d(opacity, mean, log_scale).
"""
from __future__ import annotations

import torch

from .tracer import Gaussians, TraceParams, build_bvh, trace_visibility, trace_visibility_backward


class VisibilityFn(torch.autograd.Function):
    """(vis_mean [n], vis_ray [n, K]) = VisibilityFn.apply(opacity, mean, log_scale, quat, normal, dirs, params)."""

    @staticmethod
    def forward(ctx, opacity, mean, log_scale, quat, normal, dirs, params):
        params = params or TraceParams()
        g = Gaussians(mean.detach(), quat.detach(), log_scale.detach(), opacity.detach(),
                      None if normal is None else normal.detach(), device=mean.device)
        bvh = build_bvh(g)
        vis_ray, vis_mean = trace_visibility(bvh, g, dirs, params, want_ray=True, want_mean=True)
        ctx.set_materialize_grads(False)
        ctx.bvh, ctx.g, ctx.dirs, ctx.params = bvh, g, dirs, params
        ctx.save_for_backward(vis_ray)
        return vis_mean, vis_ray

    @staticmethod
    def backward(ctx, grad_mean, grad_ray):
        (vis_ray,) = ctx.saved_tensors
        if grad_mean is None and grad_ray is None:
            return (None,) * 7
        go, gm, gl = trace_visibility_backward(ctx.bvh, ctx.g, ctx.dirs, ctx.params, grad_vis_ray=grad_ray,
                                               grad_vis_mean=grad_mean, vis_ray_fwd=vis_ray)
        return go, gm, gl, None, None, None, None


def visibility(opacity, mean, log_scale, quat, normal, dirs, params: TraceParams | None = None):
    return VisibilityFn.apply(opacity, mean, log_scale, quat, normal, dirs, params)
