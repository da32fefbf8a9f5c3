"""Python layer over the surrogate entry points of the C ABI (marshalling only)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from .tracer import BVH, Gaussians, TraceParams, _alloc_bytes, _dirs, _stream_ptr, check_pair

_F32 = torch.float32


def n_params() -> int:
    return int(_lib.load().rv_surrogate_n_params())


def _vec3(t, name, dev):
    t = torch.as_tensor(t).to(device=dev, dtype=_F32).contiguous()
    if t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{name} must be [n, 3]")
    return t


class Surrogate:
    """Parameter blob of the MLP visibility surrogate (FP32 master, Adam state, BF16 copies)."""

    def __init__(self, box_lo, box_hi, seed: int = 0, init_weights=None, device="cuda"):
        L = _lib.load()
        self.device = torch.device(device)
        self.blob = _alloc_bytes(L.rv_surrogate_bytes(), self.device)
        lo = (C.c_float * 3)(*[float(v) for v in box_lo])
        hi = (C.c_float * 3)(*[float(v) for v in box_hi])
        w = None
        if init_weights is not None:
            w = torch.as_tensor(init_weights, dtype=_F32).to(self.device).contiguous()
            if w.numel() != n_params():
                raise ValueError(f"init_weights must have {n_params()} elements")
        self.step = 0
        _lib.call("rv_surrogate_init", self.blob.data_ptr(), int(seed), lo, hi, None if w is None else w.data_ptr(),
                  _stream_ptr(self.device))
        self._train_ws = None

    def _view(self, attr, count):
        v = _lib.RvSurrogateArrays()
        _lib.call("rv_surrogate_view", self.blob.data_ptr(), C.byref(v))
        off = getattr(v, attr) - self.blob.data_ptr()
        return self.blob[off:off + 4 * count].view(_F32)

    @property
    def master(self) -> torch.Tensor:
        """FP32 weights (a view into the blob), flat order W1, b1, ..., W5, b5."""
        return self._view("master", n_params())

    @property
    def adam_m(self) -> torch.Tensor:
        return self._view("adam_m", n_params())

    @property
    def adam_v(self) -> torch.Tensor:
        return self._view("adam_v", n_params())

    @property
    def header(self) -> torch.Tensor:
        return self._view("header", 16)

    def _ws(self, batch: int) -> torch.Tensor:
        need = _lib.load().rv_surrogate_train_workspace_bytes(int(batch))
        if self._train_ws is None or self._train_ws.numel() < need:
            self._train_ws = _alloc_bytes(need, self.device)
        return self._train_ws

    def loss_grad(self, x, d, T):
        """(mean loss, FP32 gradient [n_params]) on the given samples (deterministic)."""
        x, d = _vec3(x, "x", self.device), _vec3(d, "d", self.device)
        T = torch.as_tensor(T).to(device=self.device, dtype=_F32).contiguous().reshape(-1)
        n = int(T.shape[0])
        ws = self._ws(n)
        grad = torch.empty(n_params(), dtype=_F32, device=self.device)
        loss = torch.empty(1, dtype=_F32, device=self.device)
        _lib.call("rv_surrogate_loss_grad", self.blob.data_ptr(), x.data_ptr(), d.data_ptr(), T.data_ptr(), n,
                  grad.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(self.device))
        return loss, grad

    def train(self, x, d, T, steps: int, batch: int = 16384, lr: float = 1e-3, lr_min: float = 1e-5,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, seed: int = 0,
              total_steps: int | None = None) -> torch.Tensor:
        """Adam steps on batches drawn from (x, d, T); returns the per-step mean losses."""
        x, d = _vec3(x, "x", self.device), _vec3(d, "d", self.device)
        T = torch.as_tensor(T).to(device=self.device, dtype=_F32).contiguous().reshape(-1)
        ws = self._ws(batch)
        log = torch.empty(max(int(steps), 1), dtype=_F32, device=self.device)
        opts = _lib.RvTrainOpts(int(steps), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                                float(lr_min), int(seed), int(self.step),
                                int(total_steps if total_steps is not None else self.step + steps))
        _lib.call("rv_surrogate_train", self.blob.data_ptr(), x.data_ptr(), d.data_ptr(), T.data_ptr(),
                  int(T.shape[0]), C.byref(opts), log.data_ptr(), ws.data_ptr(), ws.numel(),
                  _stream_ptr(self.device))
        self.step += int(steps)
        return log[:steps]

    def infer_xd(self, x, d):
        x, d = _vec3(x, "x", self.device), _vec3(d, "d", self.device)
        n = int(x.shape[0])
        vis = torch.empty(n, dtype=_F32, device=self.device)
        unc = torch.empty(n, dtype=_F32, device=self.device)
        _lib.call("rv_surrogate_infer_xd", self.blob.data_ptr(), x.data_ptr(), d.data_ptr(), n, vis.data_ptr(),
                  unc.data_ptr(), _stream_ptr(self.device))
        return vis, unc

    def infer_grid(self, g: Gaussians, dirs, params: TraceParams | None = None, q_begin: int = 0,
                   q_count: int | None = None, tau: float = float("inf"), bvh: BVH | None = None,
                   out_vis: torch.Tensor | None = None, out_unc: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None):
        """(vis, unc, n_fallback) over queries q = i*K + k in [q_begin, q_begin + q_count)."""
        if bvh is not None:
            check_pair(bvh, g, "Surrogate.infer_grid")
        params = params or TraceParams()
        d = _dirs(dirs, self.device)
        K = int(d.shape[0])
        if q_count is None:
            q_count = g.n * K - q_begin
        vis = out_vis if out_vis is not None else torch.empty(q_count, dtype=_F32, device=self.device)
        unc = out_unc if out_unc is not None else torch.empty(q_count, dtype=_F32, device=self.device)
        nfb = torch.zeros(1, dtype=torch.int64, device=self.device)
        need = _lib.load().rv_surrogate_infer_workspace_bytes(int(q_count))
        if workspace is None or workspace.numel() < need:
            workspace = _alloc_bytes(need, self.device)
        gc, pc = g.c(), params.c()
        _lib.call("rv_surrogate_infer", self.blob.data_ptr(), None if bvh is None else bvh.ptr, C.byref(gc),
                  d.data_ptr(), K, C.byref(pc), int(q_begin), int(q_count), float(tau), vis.data_ptr(),
                  unc.data_ptr(), nfb.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream_ptr(self.device))
        return vis, unc, nfb


def ray_setup(g: Gaussians, dirs, ray_ids, params: TraceParams | None = None):
    """(origins [n,3], unit directions [n,3]) of ray ids r = i*K + k, as the tracer forms them."""
    params = params or TraceParams()
    dev = g.mean.device
    d = _dirs(dirs, dev)
    ids = torch.as_tensor(ray_ids, dtype=torch.int64).to(dev).contiguous()
    n = int(ids.shape[0])
    o = torch.empty((n, 3), dtype=_F32, device=dev)
    dd = torch.empty((n, 3), dtype=_F32, device=dev)
    gc, pc = g.c(), params.c()
    _lib.call("rv_ray_setup", C.byref(gc), d.data_ptr(), int(d.shape[0]), C.byref(pc), ids.data_ptr(), n,
              o.data_ptr(), dd.data_ptr(), _stream_ptr(dev))
    return o, dd
