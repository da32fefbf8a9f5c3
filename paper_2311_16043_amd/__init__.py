"""MI355X (gfx950) point-based ray tracing of 3D Gaussians.

Implements the visibility pre-computation of "Relightable 3D Gaussians"
(arXiv 2311.16043), Sec. 4, as hand-written HIP kernels behind a C ABI
(include/rvis.h, librvis.so). This package is the thin Python layer: PyTorch
provides device memory and streams only.
"""
from ._lib import RvError, load  # noqa: F401
from .tracer import (BVH, Gaussians, TraceParams, build_bvh, refit_bvh, trace_rays, trace_stats,  # noqa: F401
                     trace_visibility, trace_visibility_backward, trace_visibility_sh, stream_copy,
                     gather_probe, stream_read)
from .autograd import VisibilityFn, visibility  # noqa: F401
from .surrogate import Surrogate, ray_setup  # noqa: F401
from .shading import shade_pbr  # noqa: F401
