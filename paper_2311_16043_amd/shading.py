"""Python layer over rv_shade_pbr (marshalling only): per-Gaussian PBR colour
from pre-computed visibility (Sec. 3.3, Eq. (7)-(10))."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .tracer import Gaussians, TraceParams, _dirs, _stream_ptr

_F32 = torch.float32


def shade_pbr(g: Gaussians, dirs, vis_ray: torch.Tensor, albedo, roughness, sh, env, camera, f0: float = 0.04,
              params: TraceParams | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """color [n, 3] of every Gaussian: albedo [n,3], roughness [n], sh [n,9,3],
    env [16,32,3], camera (3,), vis_ray [n, K] for the directions dirs."""
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    K = int(d.shape[0])

    def dev32(t, shape, name):
        t = torch.as_tensor(t).to(device=dev, dtype=_F32).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        return t

    vis = dev32(vis_ray, (g.n, K), "vis_ray")
    alb = dev32(albedo, (g.n, 3), "albedo")
    rough = dev32(roughness, (g.n,), "roughness")
    shc = dev32(sh, (g.n, 9, 3), "sh")
    envm = dev32(env, (16, 32, 3), "env")
    color = out if out is not None else torch.empty((g.n, 3), dtype=_F32, device=dev)
    cam = [float(v) for v in camera]
    m = _lib.RvPbrMaterial(alb.data_ptr(), rough.data_ptr(), shc.data_ptr(), envm.data_ptr(),
                           (C.c_float * 3)(*cam), float(f0))
    gc, pc = g.c(), params.c()
    _lib.call("rv_shade_pbr", C.byref(gc), d.data_ptr(), K, C.byref(pc), vis.data_ptr(), C.byref(m),
              color.data_ptr(), _stream_ptr(dev))
    return color
