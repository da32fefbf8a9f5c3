"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, answers size queries, and rejects invalid arguments before touching
the device (these calls never launch anything, so they run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2311_16043_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_16043_amd import build
        build.build(verbose=False)
    return _lib.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rvis.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rv_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.SIGNATURES), "binding signatures must cover the header exactly"


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.rv_version()


def test_size_queries(lib):
    assert lib.rv_bvh_bytes(0) == 0
    prev = 0
    for n in (1, 2, 1000, 300_000, 3_000_000):
        b = lib.rv_bvh_bytes(n)
        assert b % 256 == 0 and b >= prev
        # at least keys, perm, nodes, leaf records
        assert b >= n * (8 + 4 + 64) + (n - 1) * 64
        prev = b
        assert lib.rv_build_workspace_bytes(n) >= n * 12


def test_bvh_view_offsets_are_aligned_and_ordered(lib):
    base = 1 << 40  # never dereferenced
    out = _lib.RvBvhArrays()
    assert lib.rv_bvh_view(base, 1000, C.byref(out)) == 0
    ptrs = [out.header, out.keys, out.perm, out.nodes, out.parent, out.leaf_records, out.leaf_boxes, out.origins,
            out.nodes4]
    assert all(p % 256 == 0 for p in ptrs)
    assert ptrs == sorted(ptrs) and ptrs[0] == base
    assert ptrs[-1] + 999 * 64 <= base + lib.rv_bvh_bytes(1000)
    assert lib.rv_bvh_view(None, 10, C.byref(out)) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_bvh_view(base, 0, C.byref(out)) == _lib.RV_ERR_INVALID_ARG


def _g(n=10, ptr=1 << 40, normal=True):
    return _lib.RvGaussians(ptr, ptr, ptr, ptr, ptr if normal else None, n)


def test_build_rejects_bad_arguments(lib):
    g = _g()
    ok_bytes = lib.rv_bvh_bytes(10)
    ws = lib.rv_build_workspace_bytes(10)
    P = 1 << 40
    assert lib.rv_build_bvh(None, P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert b"null" in lib.rv_last_error()
    assert lib.rv_build_bvh(C.byref(_g(0)), P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_build_bvh(C.byref(_g(1 << 31)), P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_build_bvh(C.byref(g), P + 4, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_build_bvh(C.byref(g), P, ok_bytes - 256, P, ws, None) == _lib.RV_ERR_WORKSPACE
    assert lib.rv_build_bvh(C.byref(g), P, ok_bytes, P, ws - 256, None) == _lib.RV_ERR_WORKSPACE
    bad = _g()
    bad.quat = None
    assert lib.rv_build_bvh(C.byref(bad), P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG


def _params(**kw):
    p = dict(alpha_min=1 / 255, alpha_max=0.99, T_min=1e-4, sigma_cut=3.0, tmin_scale=3.0, dir_mode=1)
    p.update(kw)
    return _lib.RvTraceParams(**p)


@pytest.mark.parametrize("bad", [dict(dir_mode=2), dict(sigma_cut=3.5), dict(sigma_cut=0.0), dict(alpha_max=1.0),
                                 dict(alpha_min=0.0), dict(T_min=-1.0), dict(T_min=1.0), dict(alpha_min=0.995)])
def test_trace_rejects_bad_params(lib, bad):
    P = 1 << 40
    g = _g()
    p = _params(**bad)
    ws = lib.rv_trace_workspace_bytes(10, 8)
    assert lib.rv_trace_visibility(P, C.byref(g), P, 8, C.byref(p), P, P, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_last_error()


def test_trace_rejects_bad_arguments(lib):
    P = 1 << 40
    g = _g()
    p = _params()
    f = lib.rv_trace_visibility
    ws = lib.rv_trace_workspace_bytes(10, 8)
    assert ws >= 256 + 10 * 8 * 4 and ws % 256 == 0
    assert f(P, C.byref(g), P, 0, C.byref(p), P, P, P, ws, None) == _lib.RV_ERR_INVALID_ARG  # K = 0
    assert f(P, C.byref(g), P, 8, C.byref(p), None, None, P, ws, None) == _lib.RV_ERR_INVALID_ARG  # no output
    assert f(None, C.byref(g), P, 8, C.byref(p), P, P, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    gn = _g(normal=False)
    assert f(P, C.byref(gn), P, 8, C.byref(p), P, P, P, ws, None) == _lib.RV_ERR_INVALID_ARG  # hemisphere, no normal
    # the workspace: always needed (queue counters), 256 bytes with per-ray output, the full size without
    assert f(P, C.byref(g), P, 8, C.byref(p), P, P, None, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(P, C.byref(g), P, 8, C.byref(p), P, P, P + 64, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(P, C.byref(g), P, 8, C.byref(p), P, P, P, 255, None) == _lib.RV_ERR_WORKSPACE
    assert f(P, C.byref(g), P, 8, C.byref(p), None, P, P, ws - 256, None) == _lib.RV_ERR_WORKSPACE
    assert lib.rv_trace_rays(P, C.byref(g), P, 8, C.byref(p), P, -1, P, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_trace_rays(P, C.byref(g), P, 8, C.byref(p), None, 0, None, None) == 0  # empty list: no-op
    assert lib.rv_trace_visibility_backward(P, C.byref(g), P, 8, C.byref(p), None, None, None, P, P, P,
                                            None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_trace_visibility_backward(P, C.byref(g), P, 8, C.byref(p), P, None, None, None, P, P,
                                            None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_trace_stats(P, C.byref(g), P, 8, C.byref(p), None, P, 256, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_trace_stats(P, C.byref(g), P, 8, C.byref(p), P, None, 0, None) == _lib.RV_ERR_INVALID_ARG
    assert lib.rv_trace_stats(P, C.byref(g), P, 8, C.byref(p), P, P, 128, None) == _lib.RV_ERR_WORKSPACE


def test_refit_rejects_bad_arguments(lib):
    P = 1 << 40
    g = _g()
    ok_bytes = lib.rv_bvh_bytes(10)
    ws = lib.rv_build_workspace_bytes(10)
    f = lib.rv_refit_bvh
    assert f(None, P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(g), None, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(g), P, ok_bytes, None, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(_g(0)), P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(g), P + 8, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(g), P, ok_bytes - 256, P, ws, None) == _lib.RV_ERR_WORKSPACE
    assert f(C.byref(g), P, ok_bytes, P, ws - 256, None) == _lib.RV_ERR_WORKSPACE
    bad = _g()
    bad.opacity = None
    assert f(C.byref(bad), P, ok_bytes, P, ws, None) == _lib.RV_ERR_INVALID_ARG


def test_sh_workspace_and_rejects_bad_arguments(lib):
    assert lib.rv_trace_sh_workspace_bytes(0, 8) == 0
    assert lib.rv_trace_sh_workspace_bytes(10, 0) == 0
    prev = 0
    for n, K in ((1, 1), (10, 8), (1000, 256), (300_000, 256), (3_000_000, 1024)):
        b = lib.rv_trace_sh_workspace_bytes(n, K)
        # queue counters, the K x 9 table and one batch of per-ray values
        # (all n rows up to 2^28 values, never more than 2^28 + a table)
        rows = min(n * K, 1 << 28)
        assert b % 256 == 0 and b >= 256 + K * 9 * 4 + rows * 4 and b >= prev
        assert b <= 256 + K * 9 * 4 + (1 << 28) * 4 + 1024
        prev = b
    P = 1 << 40
    g = _g()
    p = _params()
    ws = lib.rv_trace_sh_workspace_bytes(10, 8)
    f = lib.rv_trace_visibility_sh
    assert f(P, C.byref(g), P, 8, C.byref(p), None, None, P, ws, None) == _lib.RV_ERR_INVALID_ARG  # no vis_sh
    assert f(P, C.byref(g), P, 0, C.byref(p), P, None, P, ws, None) == _lib.RV_ERR_INVALID_ARG  # K = 0
    assert f(P, C.byref(g), P, 8, C.byref(p), P, None, None, ws, None) == _lib.RV_ERR_INVALID_ARG  # no ws
    assert f(P, C.byref(g), P, 8, C.byref(p), P, None, P + 16, ws, None) == _lib.RV_ERR_INVALID_ARG  # unaligned
    assert f(P, C.byref(g), P, 8, C.byref(p), P, None, P, ws - 256, None) == _lib.RV_ERR_WORKSPACE
    bad = _params(dir_mode=3)
    assert f(P, C.byref(g), P, 8, C.byref(bad), P, None, P, ws, None) == _lib.RV_ERR_INVALID_ARG


def _material(**kw):
    P = 1 << 40
    m = _lib.RvPbrMaterial(P, P, P, P, (C.c_float * 3)(0.0, 0.0, 3.0), 0.04)
    for k, v in kw.items():
        if k == "camera":
            m.camera = (C.c_float * 3)(*v)
        else:
            setattr(m, k, v)
    return m


@pytest.mark.parametrize("bad", [dict(albedo=None), dict(roughness=None), dict(sh=None), dict(env=None),
                                 dict(f0=-0.1), dict(f0=1.5), dict(f0=float("nan")),
                                 dict(camera=(0.0, float("inf"), 1.0)), dict(camera=(float("nan"), 0.0, 1.0))])
def test_shade_rejects_bad_material(lib, bad):
    P = 1 << 40
    g = _g()
    p = _params()
    m = _material(**bad)
    assert lib.rv_shade_pbr(C.byref(g), P, 8, C.byref(p), P, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG
    assert b"rv_shade_pbr" in lib.rv_last_error()


def test_shade_rejects_bad_arguments(lib):
    P = 1 << 40
    g = _g()
    p = _params()
    m = _material()
    f = lib.rv_shade_pbr
    assert f(None, P, 8, C.byref(p), P, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(g), P, 0, C.byref(p), P, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG  # K = 0
    assert f(C.byref(g), P, 8, C.byref(p), None, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG  # no vis
    assert f(C.byref(g), P, 8, C.byref(p), P, None, P, None) == _lib.RV_ERR_INVALID_ARG  # no material
    assert f(C.byref(g), P, 8, C.byref(p), P, C.byref(m), None, None) == _lib.RV_ERR_INVALID_ARG  # no output
    assert f(C.byref(_g(normal=False)), P, 8, C.byref(p), P, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG
    assert f(C.byref(_g(0)), P, 8, C.byref(p), P, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG
    bad = _params(dir_mode=2)
    assert f(C.byref(g), P, 8, C.byref(bad), P, C.byref(m), P, None) == _lib.RV_ERR_INVALID_ARG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()


def test_wrappers_reject_a_tree_of_another_gaussian_set():
    """Every Python entry point that takes a BVH checks that it was built over
    a Gaussian set of the same size before calling the library (the C ABI
    derives the blob's section offsets from g.n)."""
    import numpy as np
    import torch

    from paper_2311_16043_amd import (BVH, Gaussians, Surrogate, refit_bvh, trace_rays, trace_stats,
                                      trace_visibility, trace_visibility_backward, trace_visibility_sh)
    n = 10
    g = Gaussians(np.zeros((n, 3), np.float32), np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                  np.full((n, 3), -3.0, np.float32), np.full(n, 0.5, np.float32),
                  np.tile(np.float32([0, 0, 1]), (n, 1)), device="cpu")
    bvh = BVH(torch.empty(0, dtype=torch.uint8), n + 1)
    dirs = np.float32([[0, 0, 1]])
    calls = [lambda: trace_visibility(bvh, g, dirs), lambda: trace_visibility_sh(bvh, g, dirs),
             lambda: trace_rays(bvh, g, dirs, [0]), lambda: trace_stats(bvh, g, dirs),
             lambda: trace_visibility_backward(bvh, g, dirs, grad_vis_mean=torch.zeros(n)),
             lambda: refit_bvh(bvh, g)]
    for call in calls:
        with pytest.raises(ValueError, match="built over 11 Gaussians"):
            call()
    net = Surrogate.__new__(Surrogate)  # no blob needed: the check comes first
    net.device = torch.device("cpu")
    with pytest.raises(ValueError, match="built over 11 Gaussians"):
        net.infer_grid(g, dirs, bvh=bvh)


def _opts(**kw):
    o = dict(steps=1, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, lr_min=1e-5, seed=0, step0=0,
             total_steps=1)
    o.update(kw)
    return _lib.RvTrainOpts(**o)


def test_surrogate_rejects_bad_arguments(lib):
    P = 1 << 40
    INV, WS = _lib.RV_ERR_INVALID_ARG, _lib.RV_ERR_WORKSPACE
    assert lib.rv_surrogate_init(None, 0, P, P, None, None) == INV
    assert lib.rv_surrogate_init(P + 16, 0, P, P, None, None) == INV   # blob not 256-byte aligned
    ws = lib.rv_surrogate_train_workspace_bytes(256)
    assert ws > 0 and ws % 256 == 0
    tr = lib.rv_surrogate_train
    assert tr(None, P, P, P, 100, C.byref(_opts()), P, P, ws, None) == INV
    assert tr(P, P, P, P, 0, C.byref(_opts()), P, P, ws, None) == INV          # no samples
    for bad in (dict(steps=-1), dict(batch=0), dict(batch=100), dict(lr=-1.0), dict(beta1=1.0), dict(beta2=1.0),
                dict(beta1=-0.1), dict(eps=0.0)):
        assert tr(P, P, P, P, 100, C.byref(_opts(**bad)), P, P, ws, None) == INV, bad
    assert tr(P, P, P, P, 100, C.byref(_opts()), P, P + 64, ws, None) == INV    # workspace not aligned
    assert tr(P, P, P, P, 100, C.byref(_opts()), P, P, ws - 256, None) == WS
    lg = lib.rv_surrogate_loss_grad
    assert lg(P, P, P, P, 0, P, P, P, ws, None) == INV
    assert lg(P, P, P, P, (1 << 30) + 1, P, P, P, ws, None) == INV
    assert lg(P, P, P, P, 256, P, P, P, ws - 256, None) == WS
    xd = lib.rv_surrogate_infer_xd
    assert xd(P, P, P, -1, P, None, None) == INV
    assert xd(P, None, P, 4, P, None, None) == INV
    assert xd(P, None, None, 0, P, None, None) == 0                            # n = 0: no-op
    g, p = _g(), _params()
    inf = lib.rv_surrogate_infer
    need = lib.rv_surrogate_infer_workspace_bytes(80)
    assert need % 256 == 0 and need >= 256 + 80 * 9
    assert inf(P, None, None, P, 8, C.byref(p), 0, 80, 0.1, P, None, None, P, need, None) == INV
    assert inf(P, None, C.byref(g), P, 0, C.byref(p), 0, 80, 0.1, P, None, None, P, need, None) == INV   # K = 0
    assert inf(P, None, C.byref(_g(1 << 31)), P, 8, C.byref(p), 0, 80, 0.1, P, None, None, P, need,
               None) == INV                                                   # n beyond RV_MAX_GAUSSIANS
    assert inf(P, None, C.byref(_g(normal=False)), P, 8, C.byref(p), 0, 80, 0.1, P, None, None, P, need,
               None) == INV                                                   # hemisphere without normals
    assert inf(P, None, C.byref(g), P, 8, C.byref(_params(sigma_cut=4.0)), 0, 80, 0.1, P, None, None, P, need,
               None) == INV
    assert inf(P, None, C.byref(g), P, 8, C.byref(p), 1, 80, 0.1, P, None, None, P, need, None) == INV   # past n K
    assert inf(P, None, C.byref(g), P, 8, C.byref(p), -1, 10, 0.1, P, None, None, P, need, None) == INV
    assert inf(P, None, C.byref(g), P, 8, C.byref(p), 0, 80, 0.1, P, None, None, None, need, None) == INV
    assert inf(P, None, C.byref(g), P, 8, C.byref(p), 0, 80, 0.1, P, None, None, P + 64, need, None) == INV
    assert inf(P, None, C.byref(g), P, 8, C.byref(p), 0, 80, 0.1, P, None, None, P, need - 256, None) == WS
    assert inf(P, None, C.byref(g), P, 8, C.byref(p), 80, 0, 0.1, P, None, None, None, 0, None) == 0  # empty range
    assert lib.rv_last_error() is not None


def test_ray_setup_rejects_bad_arguments(lib):
    P = 1 << 40
    INV = _lib.RV_ERR_INVALID_ARG
    g, p = _g(), _params()
    f = lib.rv_ray_setup
    assert f(None, P, 8, C.byref(p), P, 4, P, P, None) == INV
    assert f(C.byref(g), P, 0, C.byref(p), P, 4, P, P, None) == INV             # K = 0
    assert f(C.byref(g), P, 8, C.byref(p), P, -1, P, P, None) == INV            # n < 0
    assert f(C.byref(_g(0)), P, 8, C.byref(p), P, 4, P, P, None) == INV
    assert f(C.byref(_g(1 << 31)), P, 8, C.byref(p), P, 4, P, P, None) == INV
    assert f(C.byref(_g(normal=False)), P, 8, C.byref(p), P, 4, P, P, None) == INV
    assert f(C.byref(g), P, 8, C.byref(p), None, 4, P, P, None) == INV          # no ids
    assert f(C.byref(g), P, 8, C.byref(p), P, 4, P, None, None) == INV          # no output
    assert f(C.byref(g), P, 8, C.byref(p), None, 0, None, None, None) == 0      # n = 0: no-op
