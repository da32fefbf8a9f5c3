"""The largest sizes: inference over more than 2^31 queries (split into
several grids, since a dispatch counts its work-items in 32 bits), an all-ray
trace over more than 2^32 rays (one persistent grid whose pool indices pass
2^32 rays' worth, with the rows of the means in an 18 GB workspace), and the
surrogate-scale workload (3M Gaussians x 1,024 directions) against the FP64
oracle. Every output is written and equal to what the single-ray entry points
give for the same rays."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_16043_amd import Gaussians, Surrogate, TraceParams, build_bvh, ray_setup, trace_rays, trace_visibility
from workloads import scenes

from _parity import check_vis

pytestmark = pytest.mark.gpu


def test_surrogate_grid_beyond_2_31_queries():
    n, K = 2_200_000, 1024                      # 2.25e9 queries > 2^31
    print(f"[large] surrogate grid n={n} K={K}", flush=True)
    sc = scenes.make_cube_cloud(n, 0)
    dirs = scenes.fibonacci_dirs(K, False)
    prm = TraceParams(dir_mode=0)
    g = Gaussians.from_scene(sc)
    net = Surrogate(sc["mean"].min(0), sc["mean"].max(0), seed=5)
    Q = n * K
    vis = torch.full((Q,), float("nan"), dtype=torch.float32, device="cuda")
    unc = torch.full((Q,), float("nan"), dtype=torch.float32, device="cuda")
    net.infer_grid(g, dirs, prm, tau=float("inf"), out_vis=vis, out_unc=unc)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(vis).any()) and not bool(torch.isnan(unc).any()), "unwritten outputs"
    # queries on both sides of 2^31 and at the very end, against the free-form entry point
    rng = np.random.default_rng(4)
    ids = np.concatenate([rng.integers(0, Q, 2048), np.arange(2**31 - 64, 2**31 + 64), np.arange(Q - 64, Q)])
    o, d = ray_setup(g, dirs, ids, prm)
    vx, ux = net.infer_xd(o, d)
    sel = torch.from_numpy(ids).cuda()
    assert torch.equal(vx, vis[sel]) and torch.equal(ux, unc[sel])
    del vis, unc


def test_trace_beyond_2_32_lane_rays():
    n, K = 4_400_000, 1024                      # 4.5e9 rays
    print(f"[large] trace n={n} K={K}", flush=True)
    sc = scenes.make_cube_cloud(n, 0)
    dirs = scenes.fibonacci_dirs(K, False)
    prm = TraceParams(dir_mode=0)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    _, vm = trace_visibility(bvh, g, dirs, prm, want_ray=False)
    torch.cuda.synchronize()
    # Gaussians first and last in sorted order (the first and the last XCD
    # queue) and a random sample: their means from the ray-list kernel
    perm = bvh.arrays()["perm"].astype(np.int64)
    sample = np.concatenate([perm[:64], perm[-64:], np.random.default_rng(2).integers(0, n, 64)])
    ids = (sample[:, None] * K + np.arange(K)[None, :]).reshape(-1)
    T = trace_rays(bvh, g, dirs, ids, prm).cpu().numpy().astype(np.float64).reshape(-1, K)
    want = (T.sum(1) / K).astype(np.float32)
    got = vm.cpu().numpy()[sample]
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - want) <= 2 * np.spacing(np.abs(want))), np.abs(got - want).max()


def test_surrogate_scale_full_size_sampled():
    """3M Gaussians (20 objects) x 1,024 hemisphere directions, traced as the
    bench traces it (the all-ray kernel writing all 3.07e9 rays); 16,384 seeded
    rays of that output against the brute-force FP64 oracle, the ray-list
    kernel giving them the same bits, and the means of 8 Gaussians against
    their 1,024 rays."""
    sc = scenes.make_scene("surrogate")
    dirs = scenes.preset_dirs("surrogate")
    n, K = sc["mean"].shape[0], dirs.shape[0]
    print(f"[large] surrogate scale n={n} K={K}", flush=True)
    prm = TraceParams()
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    vr_all, vm = trace_visibility(bvh, g, dirs, prm)
    ids = scenes.sample_ray_ids(n, K, 16384, seed=17)
    sample = np.random.default_rng(18).integers(0, n, 8)
    rows = (sample[:, None] * K + np.arange(K)[None, :]).reshape(-1)
    flat = vr_all.reshape(-1)
    vr = flat[torch.from_numpy(ids).cuda()].cpu().numpy()
    row_vals = flat[torch.from_numpy(rows).cuda()].cpu().numpy()
    del vr_all, flat
    lst = trace_rays(bvh, g, dirs, ids, prm).cpu().numpy()
    assert np.array_equal(lst.view(np.uint32), vr.view(np.uint32))
    print(f"[large] oracle on {ids.size} rays", flush=True)
    orc = oracle.trace_rays(sc, dirs, 1, ids, oracle.params(alpha_min=1 / 255, alpha_max=0.99,
                                                            sigma_cut=prm.sigma_cut, tmin_scale=prm.tmin_scale))
    check_vis(vr, orc, label="surrogate-scale sampled")
    T = row_vals.astype(np.float64).reshape(-1, K)
    want = (T.sum(1) / K).astype(np.float32)
    got = vm.cpu().numpy()[sample]
    assert np.all(np.abs(got - want) <= 2 * np.spacing(np.abs(want))), np.abs(got - want).max()
