"""Python API over the C ABI: BVH build, visibility tracing, statistics, adjoint.

PyTorch only provides device memory and the stream; every step of the path
runs in the HIP kernels of librvis.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

_F32 = torch.float32


@dataclass
class TraceParams:
    """Cut parameters (Sec. 4.1 early termination T_min; alpha cut/clamp,
    3-sigma support and t_min = tmin_scale * max scale of the source)."""
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    sigma_cut: float = 3.0
    tmin_scale: float = 3.0
    dir_mode: int = 1  # 0: world-frame sphere directions, 1: hemisphere about the normal

    def c(self) -> _lib.RvTraceParams:
        return _lib.RvTraceParams(self.alpha_min, self.alpha_max, self.T_min, self.sigma_cut,
                                  self.tmin_scale, int(self.dir_mode))


def _dev(t, shape_tail, name, device) -> torch.Tensor:
    t = torch.as_tensor(t)
    if t.dtype != _F32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    t = t.to(device)
    if not t.is_contiguous():
        t = t.contiguous()
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}], got {tuple(t.shape)}")
    return t


class Gaussians:
    """Device-resident geometric Gaussian set (FP32, contiguous)."""

    def __init__(self, mean, quat, log_scale, opacity, normal=None, device="cuda"):
        self.mean = _dev(mean, (3,), "mean", device)
        self.quat = _dev(quat, (4,), "quat", device)
        self.log_scale = _dev(log_scale, (3,), "log_scale", device)
        self.opacity = _dev(torch.as_tensor(opacity).reshape(-1), (), "opacity", device)
        self.normal = None if normal is None else _dev(normal, (3,), "normal", device)
        self.n = int(self.mean.shape[0])
        for name in ("quat", "log_scale", "opacity"):
            if int(getattr(self, name).shape[0]) != self.n:
                raise ValueError(f"{name} has {getattr(self, name).shape[0]} rows, mean has {self.n}")

    @classmethod
    def from_scene(cls, scene: dict, device="cuda") -> "Gaussians":
        return cls(*(torch.from_numpy(np.ascontiguousarray(scene[k], dtype=np.float32))
                     for k in ("mean", "quat", "log_scale", "opacity", "normal")), device=device)

    def c(self) -> _lib.RvGaussians:
        p = lambda t: None if t is None else t.data_ptr()
        return _lib.RvGaussians(p(self.mean), p(self.quat), p(self.log_scale), p(self.opacity),
                                p(self.normal), self.n)


def _stream_ptr(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _alloc_bytes(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 256-byte (or better) aligned blocks
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class BVH:
    """A built LBVH: one device blob owned by a torch tensor."""

    def __init__(self, blob: torch.Tensor, n: int):
        self.blob = blob
        self.n = n

    @property
    def ptr(self) -> int:
        return self.blob.data_ptr()

    def view(self) -> _lib.RvBvhArrays:
        out = _lib.RvBvhArrays()
        _lib.call("rv_bvh_view", self.ptr, self.n, C.byref(out))
        return out

    def arrays(self) -> dict:
        """Copy the BVH sections to host numpy arrays (for tests and inspection)."""
        n = self.n
        base = self.ptr
        v = self.view()

        def grab(ptr, count, dtype):
            off = ptr - base
            nbytes = count * np.dtype(dtype).itemsize
            return self.blob[off:off + nbytes].cpu().numpy().view(dtype).copy()

        nodes = grab(v.nodes, 16 * max(n - 1, 0), np.float32).reshape(-1, 16)
        ids = nodes[:, 12:14].view(np.int32) if n > 1 else np.zeros((0, 2), np.int32)
        return dict(
            header=grab(v.header, 16, np.float32),
            keys=grab(v.keys, n, np.uint64),
            perm=grab(v.perm, n, np.uint32),
            nodes=nodes,
            left=ids[:, 0].copy(),
            right=ids[:, 1].copy(),
            left_box=nodes[:, 0:6].copy(),
            right_box=nodes[:, 6:12].copy(),
            parent=grab(v.parent, 2 * n - 1, np.int32),
            leaf_records=grab(v.leaf_records, 12 * n, np.float32).reshape(n, 12),
            leaf_boxes=grab(v.leaf_boxes, 6 * n, np.float32).reshape(n, 6),
            origins=grab(v.origins, 4 * n, np.float32).reshape(n, 4),
            nodes4=grab(v.nodes4, 16 * max(n - 1, 0), np.uint32).reshape(-1, 16),
        )


def check_pair(bvh: BVH, g: Gaussians, fn: str) -> None:
    """Raise unless `bvh` was built over a Gaussian set of g's size (the C
    ABI derives every section offset of the blob from g.n)."""
    if g.n != bvh.n:
        raise ValueError(f"{fn}: the BVH was built over {bvh.n} Gaussians, g has {g.n}; rebuild it")


def build_bvh(g: Gaussians, workspace: torch.Tensor | None = None) -> BVH:
    L = _lib.load()
    dev = g.mean.device
    blob = _alloc_bytes(L.rv_bvh_bytes(g.n), dev)
    ws_bytes = L.rv_build_workspace_bytes(g.n)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc_bytes(ws_bytes, dev)
    gc = g.c()
    _lib.call("rv_build_bvh", C.byref(gc), blob.data_ptr(), blob.numel(), workspace.data_ptr(),
              workspace.numel(), _stream_ptr(dev))
    return BVH(blob, g.n)


def _dirs(dirs, device) -> torch.Tensor:
    return _dev(torch.as_tensor(np.asarray(dirs, dtype=np.float32)) if not torch.is_tensor(dirs) else dirs,
                (3,), "dirs", device)


def refit_bvh(bvh: BVH, g: Gaussians, workspace: torch.Tensor | None = None) -> BVH:
    """Refit `bvh` in place to the (moved) Gaussians it was built from: same
    topology and order, boxes and records recomputed."""
    L = _lib.load()
    check_pair(bvh, g, "refit_bvh")
    dev = g.mean.device
    ws_bytes = L.rv_build_workspace_bytes(g.n)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc_bytes(ws_bytes, dev)
    gc = g.c()
    _lib.call("rv_refit_bvh", C.byref(gc), bvh.ptr, bvh.blob.numel(), workspace.data_ptr(), workspace.numel(),
              _stream_ptr(dev))
    return bvh


def trace_visibility(bvh: BVH, g: Gaussians, dirs, params: TraceParams | None = None,
                     want_ray: bool = True, want_mean: bool = True, out_ray: torch.Tensor | None = None,
                     out_mean: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """(vis_ray [n, K] or None, vis_mean [n] or None) for every ray (i, k)."""
    check_pair(bvh, g, "trace_visibility")
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    K = int(d.shape[0])
    vr = (out_ray if out_ray is not None else torch.empty((g.n, K), dtype=_F32, device=dev)) if want_ray else None
    vm = (out_mean if out_mean is not None else torch.empty((g.n,), dtype=_F32, device=dev)) if want_mean else None
    # 256 bytes of queue counters suffice when the per-ray values go to vr
    ws_bytes = 256 if vr is not None else _lib.load().rv_trace_workspace_bytes(g.n, K)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc_bytes(ws_bytes, dev)
    gc, pc = g.c(), params.c()
    _lib.call("rv_trace_visibility", bvh.ptr, C.byref(gc), d.data_ptr(), K, C.byref(pc),
              None if vr is None else vr.data_ptr(), None if vm is None else vm.data_ptr(), workspace.data_ptr(),
              workspace.numel(), _stream_ptr(dev))
    return vr, vm


def trace_visibility_static(bvh: BVH, g: Gaussians, dirs, params: TraceParams | None = None,
                            out_ray: torch.Tensor | None = None, out_mean: torch.Tensor | None = None):
    """trace_visibility into caller-given outputs (either may be None, not
    both), with the library's static per-device scratch instead of a
    workspace: the library call allocates nothing. Calls that overlap on one
    device race; calls on one stream are ordered."""
    check_pair(bvh, g, "trace_visibility_static")
    if out_ray is None and out_mean is None:
        raise ValueError("trace_visibility_static: give out_ray, out_mean or both")
    params = params or TraceParams()
    d = _dirs(dirs, g.mean.device)
    gc, pc = g.c(), params.c()
    _lib.call("rv_trace_visibility_static", bvh.ptr, C.byref(gc), d.data_ptr(), int(d.shape[0]), C.byref(pc),
              None if out_ray is None else out_ray.data_ptr(), None if out_mean is None else out_mean.data_ptr(),
              _stream_ptr(g.mean.device))
    return out_ray, out_mean


def trace_visibility_sh(bvh: BVH, g: Gaussians, dirs, params: TraceParams | None = None, want_mean: bool = True,
                        workspace: torch.Tensor | None = None):
    """(vis_sh [n, 9], vis_mean [n] or None): each Gaussian's visibility
    projected onto the degree-2 real SH, with no per-ray output."""
    check_pair(bvh, g, "trace_visibility_sh")
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    K = int(d.shape[0])
    sh = torch.empty((g.n, 9), dtype=_F32, device=dev)
    vm = torch.empty((g.n,), dtype=_F32, device=dev) if want_mean else None
    ws_bytes = _lib.load().rv_trace_sh_workspace_bytes(g.n, K)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc_bytes(ws_bytes, dev)
    gc, pc = g.c(), params.c()
    _lib.call("rv_trace_visibility_sh", bvh.ptr, C.byref(gc), d.data_ptr(), K, C.byref(pc), sh.data_ptr(),
              None if vm is None else vm.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream_ptr(dev))
    return sh, vm


def trace_rays(bvh: BVH, g: Gaussians, dirs, ray_ids, params: TraceParams | None = None) -> torch.Tensor:
    """T of each listed ray id r = i*K + k (same bits as trace_visibility)."""
    check_pair(bvh, g, "trace_rays")
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    ids = torch.as_tensor(ray_ids, dtype=torch.int64).to(dev).contiguous()
    out = torch.empty(ids.shape[0], dtype=_F32, device=dev)
    gc, pc = g.c(), params.c()
    _lib.call("rv_trace_rays", bvh.ptr, C.byref(gc), d.data_ptr(), int(d.shape[0]), C.byref(pc), ids.data_ptr(),
              int(ids.shape[0]), out.data_ptr(), _stream_ptr(dev))
    return out


def trace_stats(bvh: BVH, g: Gaussians, dirs, params: TraceParams | None = None) -> dict:
    """Totals over all rays: internal nodes visited, leaves tested, Gaussians included."""
    check_pair(bvh, g, "trace_stats")
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    tot = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = _alloc_bytes(256, dev)
    gc, pc = g.c(), params.c()
    _lib.call("rv_trace_stats", bvh.ptr, C.byref(gc), d.data_ptr(), int(d.shape[0]), C.byref(pc), tot.data_ptr(),
              ws.data_ptr(), ws.numel(), _stream_ptr(dev))
    t = tot.cpu().tolist()
    return dict(nodes=t[0], leaves=t[1], hits=t[2])


def trace_visibility_backward(bvh: BVH, g: Gaussians, dirs, params: TraceParams | None = None,
                              grad_vis_ray: torch.Tensor | None = None, grad_vis_mean: torch.Tensor | None = None,
                              vis_ray_fwd: torch.Tensor | None = None):
    """(grad_opacity [n], grad_mean [n,3], grad_log_scale [n,3]) of the upstream gradients."""
    check_pair(bvh, g, "trace_visibility_backward")
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    K = int(d.shape[0])

    def chk(t, shape, name):
        if t is None:
            return None
        t = t.to(device=dev, dtype=_F32).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        return t

    grad_vis_ray = chk(grad_vis_ray, (g.n, K), "grad_vis_ray")
    grad_vis_mean = chk(grad_vis_mean, (g.n,), "grad_vis_mean")
    vis_ray_fwd = chk(vis_ray_fwd, (g.n, K), "vis_ray_fwd")
    go = torch.zeros(g.n, dtype=_F32, device=dev)
    gm = torch.zeros((g.n, 3), dtype=_F32, device=dev)
    gl = torch.zeros((g.n, 3), dtype=_F32, device=dev)
    gc, pc = g.c(), params.c()
    p = lambda t: None if t is None else t.data_ptr()
    _lib.call("rv_trace_visibility_backward", bvh.ptr, C.byref(gc), d.data_ptr(), K, C.byref(pc), p(grad_vis_ray),
              p(grad_vis_mean), p(vis_ray_fwd), go.data_ptr(), gm.data_ptr(), gl.data_ptr(), _stream_ptr(dev))
    return go, gm, gl


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """dst <- src (same byte size) with the library's streaming copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: size mismatch")
    _lib.call("rv_stream_copy", src.data_ptr(), dst.data_ptr(), nbytes, _stream_ptr(src.device))


def gather_probe(table: torch.Tensor, rounds: int, blocks: int) -> torch.Tensor:
    """Record-gather probe over `table` (a device tensor of 64-byte records):
    blocks x 256 threads each read `rounds` records as three 16-byte loads at
    hashed indices. Returns the sink (one word per thread)."""
    nbytes = table.numel() * table.element_size()
    if nbytes % 64:
        raise ValueError("gather_probe: the table must hold whole 64-byte records")
    sink = torch.empty(blocks * 256, dtype=torch.int32, device=table.device)
    _lib.call("rv_gather_probe", table.data_ptr(), nbytes // 64, int(rounds), int(blocks), sink.data_ptr(),
              _stream_ptr(table.device))
    return sink


def stream_read(src: torch.Tensor) -> torch.Tensor:
    """Read src once with the library's streaming read probe; returns the sink."""
    nbytes = src.numel() * src.element_size()
    words = int(_lib.load().rv_stream_read_sink_words(nbytes))
    sink = torch.empty(words, dtype=torch.int32, device=src.device)
    _lib.call("rv_stream_read", src.data_ptr(), nbytes, sink.data_ptr(), _stream_ptr(src.device))
    return sink
