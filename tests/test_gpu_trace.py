"""GPU visibility vs the FP64 brute-force oracle (no BVH, no early exit).

Acceptance: every ray's FP32 visibility lies within 1e-4 of the oracle's
value, widened only for rays that cross a Gaussian lying within binary32
rounding of one of the cuts (t_min, 3-sigma, alpha >= 1/255); for those the
oracle returns the band [V_lo, V_hi] spanned by both decisions.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_16043_amd import Gaussians, TraceParams, build_bvh, trace_rays, trace_stats, trace_visibility
from workloads import scenes

from _parity import TOL, check_vis

pytestmark = pytest.mark.gpu


def _run(scene, dirs, params):
    g = Gaussians.from_scene(scene)
    bvh = build_bvh(g)
    vr, vm = trace_visibility(bvh, g, dirs, params)
    torch.cuda.synchronize()
    return g, bvh, vr.cpu().numpy(), vm.cpu().numpy()


def _oprm(params: TraceParams):
    return oracle.params(alpha_min=1 / 255, alpha_max=0.99, sigma_cut=params.sigma_cut,
                         tmin_scale=params.tmin_scale)


def test_tiny_all_rays_and_means():
    """2,000 Gaussians x 64 sphere directions: all 128,000 rays."""
    sc = scenes.make_scene("tiny")
    dirs = scenes.preset_dirs("tiny")
    prm = TraceParams(dir_mode=0)
    g, bvh, vr, vm = _run(sc, dirs, prm)
    n, K = vr.shape
    orc = oracle.trace_all(sc, dirs, 0, _oprm(prm))
    check_vis(vr.reshape(-1), orc, label="tiny all rays")
    # per-Gaussian mean: the band of the mean is the mean of the bands
    lo = orc["V_lo"].reshape(n, K).mean(1) - TOL
    hi = orc["V_hi"].reshape(n, K).mean(1) + TOL
    assert np.all((vm >= lo) & (vm <= hi))
    # and it is the FP64 mean of the FP32 rays, rounded
    ref = (vr.astype(np.float64).sum(1) / K).astype(np.float32)
    assert np.max(np.abs(vm - ref)) <= 1e-7


@pytest.mark.parametrize("label,maker,K,count", [
    ("object-20k", lambda: scenes.make_object_scene(20_000, 1), 32, 4096),
    ("multi-4x5000", lambda: scenes.make_multi_object_scene(4, 5_000, 2), 32, 4096),
])
def test_small_scenes_sampled(label, maker, K, count):
    sc = maker()
    dirs = scenes.fibonacci_dirs(K, True)
    prm = TraceParams()
    g, bvh, vr, vm = _run(sc, dirs, prm)
    ids = scenes.sample_ray_ids(sc["mean"].shape[0], K, count, seed=7)
    orc = oracle.trace_rays(sc, dirs, 1, ids, _oprm(prm))
    check_vis(vr.reshape(-1)[ids], orc, label=label)


def test_training_time_rotated_directions():
    """Training re-traces each iteration with the 64 directions turned about
    the normal by a fresh angle: three turns on one BVH, each against the
    oracle with the same table."""
    sc = scenes.make_object_scene(20_000, 1)
    prm = TraceParams()
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    for it, angle in enumerate((0.3, 2.1, 5.0)):
        dirs = scenes.rotated_dirs(64, angle)
        vr, _ = trace_visibility(bvh, g, dirs, prm)
        ids = scenes.sample_ray_ids(20_000, 64, 1024, seed=20 + it)
        orc = oracle.trace_rays(sc, dirs, 1, ids, _oprm(prm))
        check_vis(vr.cpu().numpy().reshape(-1)[ids], orc, label=f"rotated {angle}")


def test_object_scale_full_size_sampled():
    """300,000 Gaussians x 256 hemisphere directions, traced in full in the
    benchmark's launch configuration; 16,384 seeded rays checked."""
    sc = scenes.make_scene("object")
    dirs = scenes.preset_dirs("object")
    prm = TraceParams()
    g, bvh, vr, vm = _run(sc, dirs, prm)
    n, K = vr.shape
    ids = scenes.sample_ray_ids(n, K, 16384, seed=11)
    orc = oracle.trace_rays(sc, dirs, 1, ids, _oprm(prm))
    check_vis(vr.reshape(-1)[ids], orc, label="object-300k sampled")
    assert np.all(np.isfinite(vm)) and np.all((vm >= 0) & (vm <= 1))


def test_multi_object_full_size_sampled():
    """1.2M Gaussians x 512 hemisphere directions, every ray traced by the
    all-ray kernel; 65,536 seeded rays of its output against the oracle, and
    the ray-list kernel gives them the same bits."""
    sc = scenes.make_scene("multi")
    dirs = scenes.preset_dirs("multi")
    prm = TraceParams()
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    vr_all, vm = trace_visibility(bvh, g, dirs, prm)
    n, K = g.n, dirs.shape[0]
    ids = scenes.sample_ray_ids(n, K, 65536, seed=13)
    vr = vr_all.reshape(-1)[torch.from_numpy(ids).cuda()].cpu().numpy()
    del vr_all
    lst = trace_rays(bvh, g, dirs, ids, prm).cpu().numpy()
    assert np.array_equal(lst.view(np.uint32), vr.view(np.uint32))
    print(f"[multi-1.2M] oracle on {ids.size} rays", flush=True)
    orc = oracle.trace_rays(sc, dirs, 1, ids, _oprm(prm))
    check_vis(vr, orc, label="multi-1.2M sampled")
    vm = vm.cpu().numpy()
    assert np.all(np.isfinite(vm)) and np.all((vm >= 0) & (vm <= 1))


def test_ray_list_matches_full_trace_bitwise():
    sc = scenes.make_object_scene(30_000, 1)
    dirs = scenes.fibonacci_dirs(64, True)
    prm = TraceParams()
    g, bvh, vr, _ = _run(sc, dirs, prm)
    ids = scenes.sample_ray_ids(30_000, 64, 20_000, seed=3)
    got = trace_rays(bvh, g, dirs, ids, prm).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), vr.reshape(-1)[ids].view(np.uint32))


def test_long_ray_list_in_runs_matches_full_trace_bitwise():
    """9M listed rays: past 32,768 pools of 256, so each wave of the list kernel
    takes a run of two pools; every ray must still equal the all-ray trace."""
    sc = scenes.make_scene("object")
    dirs = scenes.preset_dirs("object")
    n, K = sc["mean"].shape[0], dirs.shape[0]
    g, bvh, vr, _ = _run(sc, dirs, TraceParams())
    ids = np.sort(np.random.default_rng(21).choice(n * K, 9_000_000, replace=False)).astype(np.int64)
    got = trace_rays(bvh, g, dirs, ids, TraceParams()).cpu().numpy()
    want = vr.reshape(-1)[ids]
    bad = int(np.count_nonzero(got.view(np.uint32) != want.view(np.uint32)))
    print(f"[long list] {ids.size} rays, mismatches {bad}", flush=True)
    assert bad == 0


def test_mean_without_per_ray_output_is_the_same():
    """Without per-ray output the rows go through the workspace; the means must
    equal those computed next to the per-ray output, bit for bit."""
    sc = scenes.make_object_scene(30_000, 1)
    dirs = scenes.fibonacci_dirs(77, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    vr, vm = trace_visibility(bvh, g, dirs)
    none, vm2 = trace_visibility(bvh, g, dirs, want_ray=False)
    torch.cuda.synchronize()
    assert none is None
    assert torch.equal(vm, vm2)
    # and they are the row means of the per-ray values
    ref = vr.double().mean(1).float()
    assert torch.max(torch.abs(vm - ref)).item() <= 1e-6


def test_trace_is_deterministic():
    sc = scenes.make_object_scene(30_000, 1)
    dirs = scenes.fibonacci_dirs(64, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    a = trace_visibility(bvh, g, dirs)
    b = trace_visibility(bvh, g, dirs)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_early_exit_changes_only_rays_below_tmin():
    """Exit once T < T_min returns the running T: for every ray
    0 <= V(T_min) - V(no exit) < T_min, and rays that never drop below T_min
    are unchanged."""
    sc = scenes.make_object_scene(30_000, 1)
    dirs = scenes.fibonacci_dirs(64, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    a, _ = trace_visibility(bvh, g, dirs, TraceParams(T_min=1e-4))
    b, _ = trace_visibility(bvh, g, dirs, TraceParams(T_min=0.0))
    a, b = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
    diff = a - b
    assert np.all(diff >= -1e-12) and np.all(diff < 1e-4)
    assert np.array_equal(a[b >= 1e-4], b[b >= 1e-4])
    assert (b < 1e-4).sum() > 1000  # the exit is exercised


def test_single_gaussian_and_single_direction():
    sc = scenes.make_cube_cloud(1, 0)
    dirs = scenes.fibonacci_dirs(8, False)
    g, bvh, vr, vm = _run(sc, dirs, TraceParams(dir_mode=0))
    assert np.all(vr == 1.0) and np.all(vm == 1.0)
    sc = scenes.make_cube_cloud(500, 0)
    dirs = scenes.fibonacci_dirs(1, False)
    g, bvh, vr, vm = _run(sc, dirs, TraceParams(dir_mode=0))
    orc = oracle.trace_all(sc, dirs, 0)
    check_vis(vr.reshape(-1), orc, label="K=1")
    assert np.array_equal(vr[:, 0], vm)


@pytest.mark.parametrize("n,K,mode", [(130, 2, 1), (70, 5, 1), (190, 3, 0), (1000, 1, 0)])
def test_fewer_pools_than_queue_ranges(n, K, mode):
    """6 to 16 pools over the eight queue ranges, ragged last groups: waves
    whose range is empty or spent take pools from the others, and lanes are
    refilled in batches from partial pools. Every ray against the oracle, and
    the ray-list kernel over all rays gives the same bits."""
    sc = scenes.make_object_scene(n, 1) if mode else scenes.make_cube_cloud(n, 0)
    dirs = scenes.fibonacci_dirs(K, bool(mode))
    prm = TraceParams(dir_mode=mode)
    g, bvh, vr, vm = _run(sc, dirs, prm)
    orc = oracle.trace_all(sc, dirs, mode, _oprm(prm))
    check_vis(vr.reshape(-1), orc, label=f"n={n} K={K}")
    ids = np.arange(n * K, dtype=np.int64)
    got = trace_rays(bvh, g, dirs, ids, prm).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), vr.reshape(-1).view(np.uint32))
    ref = (vr.astype(np.float64).sum(1) / K).astype(np.float32)
    assert np.max(np.abs(vm - ref)) <= 1e-7


def test_stats_are_consistent():
    sc = scenes.make_object_scene(20_000, 1)
    dirs = scenes.fibonacci_dirs(32, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    st = trace_stats(bvh, g, dirs)
    st2 = trace_stats(bvh, g, dirs)
    # leaf tests and inclusions are fixed by the rays; node visits made while a
    # ray's last leaves wait for the wave's leaf phase depend on scheduling
    assert st["leaves"] == st2["leaves"] and st["hits"] == st2["hits"]
    assert abs(st["nodes"] - st2["nodes"]) <= 1e-4 * st["nodes"]
    rays = 20_000 * 32
    assert st["nodes"] >= rays and st["leaves"] >= st["hits"] > 0
    # brute force tests n-1 Gaussians per ray; the BVH must test far fewer
    assert st["leaves"] < 0.05 * rays * (20_000 - 1)
    # without the early exit every included Gaussian is counted: the total
    # equals the oracle's over all rays, up to pairs binary32 may decide
    # either way (each ambiguous pair can move the count by one)
    sc = scenes.make_object_scene(3000, 2)
    dirs = scenes.fibonacci_dirs(16, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    st = trace_stats(bvh, g, dirs, TraceParams(T_min=0.0))
    orc = oracle.trace_all(sc, dirs, 1)
    incl, amb = int(orc["n_incl"].sum()), int(orc["n_amb"].sum())
    print(f"[stats] included: gpu {st['hits']}, oracle {incl}, ambiguous pairs {amb}; leaf tests {st['leaves']}",
          flush=True)
    assert abs(st["hits"] - incl) <= amb
    assert st["leaves"] >= st["hits"] > 0.5 * incl


def test_scene_far_from_the_origin():
    """Coordinates near 100: binary32 ulps are 8e-6, so box tests and leaf tests
    round much more coarsely; the result must still match the FP64 oracle."""
    sc = scenes.make_object_scene(20_000, 1)
    sc["mean"] = (sc["mean"].astype(np.float64) + np.array([97.0, -64.0, 33.0])).astype(np.float32)
    dirs = scenes.fibonacci_dirs(32, True)
    prm = TraceParams()
    g, bvh, vr, vm = _run(sc, dirs, prm)
    ids = scenes.sample_ray_ids(20_000, 32, 4096, seed=17)
    orc = oracle.trace_rays(sc, dirs, 1, ids, _oprm(prm))
    check_vis(vr.reshape(-1)[ids], orc, label="object-20k shifted")


def test_c_abi_with_a_tree_of_another_gaussian_set_gives_nan():
    """Calling the C ABI directly (past the Python check) with g.n different
    from the n the blob was built over: the kernels compare the n recorded in
    the blob's header and never walk the tree. Traces give NaN, the adjoint
    gives NaN, a refit leaves the blob as it was."""
    import ctypes as C

    from paper_2311_16043_amd import _lib
    from paper_2311_16043_amd.tracer import _stream_ptr

    sc = scenes.make_object_scene(3000, 1)
    dirs = torch.from_numpy(scenes.fibonacci_dirs(8, True)).cuda()
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    small = Gaussians.from_scene({k: v[:2000] for k, v in sc.items()})
    pc = TraceParams().c()
    gc = small.c()
    s = _stream_ptr()
    vr = torch.zeros((2000, 8), dtype=torch.float32, device="cuda")
    vm = torch.zeros(2000, dtype=torch.float32, device="cuda")
    ws = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    _lib.call("rv_trace_visibility", bvh.ptr, C.byref(gc), dirs.data_ptr(), 8, C.byref(pc), vr.data_ptr(),
              vm.data_ptr(), ws.data_ptr(), ws.numel(), s)
    ids = torch.arange(0, 2000 * 8, 7, dtype=torch.int64, device="cuda")
    out = torch.zeros(ids.numel(), dtype=torch.float32, device="cuda")
    _lib.call("rv_trace_rays", bvh.ptr, C.byref(gc), dirs.data_ptr(), 8, C.byref(pc), ids.data_ptr(), ids.numel(),
              out.data_ptr(), s)
    gmean = torch.ones(2000, dtype=torch.float32, device="cuda")
    go = torch.zeros(2000, dtype=torch.float32, device="cuda")
    gm = torch.zeros((2000, 3), dtype=torch.float32, device="cuda")
    gl = torch.zeros((2000, 3), dtype=torch.float32, device="cuda")
    _lib.call("rv_trace_visibility_backward", bvh.ptr, C.byref(gc), dirs.data_ptr(), 8, C.byref(pc), None,
              gmean.data_ptr(), None, go.data_ptr(), gm.data_ptr(), gl.data_ptr(), s)
    before = bvh.blob.clone()
    bws = torch.zeros(int(_lib.load().rv_build_workspace_bytes(2000)), dtype=torch.uint8, device="cuda")
    _lib.call("rv_refit_bvh", C.byref(gc), bvh.ptr, bvh.blob.numel(), bws.data_ptr(), bws.numel(), s)
    torch.cuda.synchronize()
    for name, t in (("vis_ray", vr), ("vis_mean", vm), ("trace_rays", out), ("grad_opacity", go),
                    ("grad_mean", gm), ("grad_log_scale", gl)):
        assert bool(torch.isnan(t).all()), name
    assert torch.equal(bvh.blob, before)
    # the blob still serves the set it was built over
    vr2, _ = trace_visibility(bvh, g, dirs)
    assert bool(torch.isfinite(vr2).all())
