"""The allocation-free variant of the all-ray trace (rv_trace_visibility_static),
called through the C ABI: its scratch is a static device array, and it must
give the bits rv_trace_visibility gives with a caller-owned workspace. Two
calls in a row, the second on a smaller input (the array keeps the first
call's contents), with per-ray output and with means only (the per-ray values
then live in the static array); a request beyond the array is refused before
anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2311_16043_amd import Gaussians, TraceParams, _lib, build_bvh
from paper_2311_16043_amd.tracer import _stream_ptr
from workloads import scenes

pytestmark = pytest.mark.gpu


def _call_static(bvh, g, dirs, prm, want_ray):
    n, K = g.n, int(dirs.shape[0])
    vr = torch.full((n, K), float("nan"), dtype=torch.float32, device="cuda") if want_ray else None
    vm = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    gc, pc = g.c(), prm.c()
    _lib.call("rv_trace_visibility_static", bvh.ptr, C.byref(gc), dirs.data_ptr(), K, C.byref(pc),
              None if vr is None else vr.data_ptr(), vm.data_ptr(), _stream_ptr())
    return vr, vm


def _call_ws(bvh, g, dirs, prm):
    n, K = g.n, int(dirs.shape[0])
    vr = torch.empty((n, K), dtype=torch.float32, device="cuda")
    vm = torch.empty((n,), dtype=torch.float32, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    gc, pc = g.c(), prm.c()
    _lib.call("rv_trace_visibility", bvh.ptr, C.byref(gc), dirs.data_ptr(), K, C.byref(pc), vr.data_ptr(),
              vm.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr())
    return vr, vm


@pytest.mark.parametrize("want_ray", [True, False])
def test_static_scratch_entry_matches_workspace_entry(want_ray):
    prm = TraceParams()
    for n, K, seed in ((20_000, 96, 1), (3_000, 17, 2)):   # the second call smaller than the first
        sc = scenes.make_object_scene(n, seed)
        dirs = torch.from_numpy(scenes.fibonacci_dirs(K, True)).cuda()
        g = Gaussians.from_scene(sc)
        bvh = build_bvh(g)
        vr_ref, vm_ref = _call_ws(bvh, g, dirs, prm)
        vr, vm = _call_static(bvh, g, dirs, prm, want_ray)
        torch.cuda.synchronize()
        print(f"[no-alloc] n={n} K={K} per-ray output {want_ray}: mean V {float(vm.mean()):.4f}", flush=True)
        if want_ray:
            assert torch.equal(vr, vr_ref), (n, K)
        assert torch.equal(vm, vm_ref), (n, K)


def test_static_scratch_entry_refuses_more_than_its_scratch():
    lib = _lib.load()
    cap = (int(lib.rv_trace_static_scratch_bytes()) - 256) // 4
    n, K = 40_000, 256                     # 10.24M rays > 8,388,544 without per-ray output
    assert n * K > cap
    sc = scenes.make_cube_cloud(n, 0)
    dirs = torch.from_numpy(scenes.fibonacci_dirs(K, False)).cuda()
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    vm = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    gc, pc = g.c(), TraceParams(dir_mode=0).c()
    st = lib.rv_trace_visibility_static(bvh.ptr, C.byref(gc), dirs.data_ptr(), K, C.byref(pc), None,
                                        vm.data_ptr(), _stream_ptr())
    assert st == -2 and b"static scratch" in lib.rv_last_error()
    torch.cuda.synchronize()
    assert bool((vm == -1.0).all())        # nothing was enqueued
