"""Benchmark: visibility rays/s of the plain BVH tracer on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload object]

A step is one pass of the hot path over the object-scale workload (300,000
surface Gaussians, 256 hemisphere directions each, 76.8M rays): LBVH build
(bounds, Morton keys, radix sort, radix tree, refit) then the traversal that
writes every ray's transmittance and each Gaussian's mean visibility. Inputs
are resident in HBM before timing starts. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


KERNEL_SOURCES = ["paper_2311_16043_amd/csrc/trace.hip", "paper_2311_16043_amd/csrc/trace_core.h",
                  "paper_2311_16043_amd/csrc/build.hip", "paper_2311_16043_amd/csrc/rv_internal.h"]
COUNTERS_FILE = "profiles/trace_object_scale_counters.md"


def recorded_traffic():
    """HBM bytes per launch from the committed counter profile, if it was taken
    on the kernel sources as they are now (else None)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        text = open(os.path.join(ROOT, COUNTERS_FILE)).read()
    except OSError:
        return None
    kv = dict(line.strip().split(": ", 1) for line in text.splitlines() if ": " in line and
              line.strip().split(": ", 1)[0] in ("kernel_sources_sha256_16", "traffic_bytes_per_launch"))
    if kv.get("kernel_sources_sha256_16") != h.hexdigest()[:16]:
        return None
    return float(kv["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="object", choices=["object", "multi", "tiny", "surrogate"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the streaming-copy probe (known-size reference for counters)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-shade", action="store_true", help="skip the PBR shading leg")
    ap.add_argument("--sur-train-samples", type=int, default=8_000_000)
    ap.add_argument("--sur-steps", type=int, default=2000)
    ap.add_argument("--sur-batch", type=int, default=16384)
    ap.add_argument("--sur-mae", type=float, default=0.02, help="target mean absolute visibility error")
    return ap.parse_args()


NODE_BYTES = 48   # compressed four-wide node: origin, exponents and kinds, 24 plane bytes, 2 child indices
LEAF_BYTES = 48   # leaf record: mean, opacity, two whitening rows, s0 s1/s2, source index
MLP_FLOPS_PER_QUERY = 2 * (64 * 256 + 3 * 256 * 256 + 256 * 2)   # dense layers, padded input width 64
BF16_PEAK_TFLOPS = 2500.0


def surrogate_leg(args, torch, g, dirs, prm, bvh, vis_ray, plain_rays_per_s):
    """Train the MLP surrogate on the tracer's samples, pick the fallback
    threshold on held-out rays, then time the surrogate path over every query."""
    from paper_2311_16043_amd import Surrogate, ray_setup
    dev = vis_ray.device
    n, K = vis_ray.shape
    R = n * K
    T_all = vis_ray.reshape(-1)
    gen = torch.Generator(device="cpu").manual_seed(2311)
    # uniform draws (a permutation of all R ids would not fit the host at the largest workload);
    # the chance that a held-out id is also a training id is train_samples / R
    tr_ids = torch.randint(R, (min(args.sur_train_samples, R),), generator=gen).to(dev)
    ho_ids = torch.randint(R, (min(1_000_000, R),), generator=gen).to(dev)
    o, d = ray_setup(g, dirs, tr_ids, prm)
    T_tr = T_all[tr_ids]
    lo = g.mean.min(0).values.cpu().tolist()
    hi = g.mean.max(0).values.cpu().tolist()
    net = Surrogate(lo, hi, seed=1, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    log = net.train(o, d, T_tr, steps=args.sur_steps, batch=args.sur_batch, lr=2e-3, lr_min=5e-5, seed=7)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    del o, d, T_tr
    # threshold: rank held-out queries by predicted error, trace the top fraction
    oh, dh = ray_setup(g, dirs, ho_ids, prm)
    vh, uh = net.infer_xd(oh, dh)
    err = (vh - T_all[ho_ids]).abs()
    order = torch.argsort(uh, descending=True)
    e_sorted = err[order]
    kept_err = torch.flip(torch.cumsum(torch.flip(e_sorted, [0]), 0), [0]) / err.numel()  # MAE if the first j are traced
    # a 5 % margin so that the error over all queries stays within the target
    ok = torch.nonzero(kept_err <= 0.95 * args.sur_mae)
    j = int(ok[0]) if ok.numel() else err.numel()
    tau = float(uh[order[j]]) if j < err.numel() else float("-inf")
    # timed: surrogate with fallback over all R queries, and the network alone
    out_v = torch.empty(R, dtype=torch.float32, device=dev)
    out_u = torch.empty(R, dtype=torch.float32, device=dev)
    ws = torch.empty(int(__import__("paper_2311_16043_amd")._lib.load().rv_surrogate_infer_workspace_bytes(R)),
                     dtype=torch.uint8, device=dev)

    def sweep(tau_, with_bvh):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, nfb = net.infer_grid(g, dirs, prm, 0, R, tau=tau_, bvh=bvh if with_bvh else None, out_vis=out_v,
                                   out_unc=out_u, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1000.0, int(nfb.item())

    sweep(float("inf"), False)
    mlp_s, _ = sweep(float("inf"), False)
    mae_net = float((out_v - T_all).abs().mean())
    fb_s, nfb = sweep(tau, True)
    mae = float((out_v - T_all).abs().mean())
    q_per_s = R / fb_s
    return dict(
        queries=R, train_samples=int(tr_ids.numel()), train_steps=args.sur_steps, batch=args.sur_batch,
        train_s=train_s, train_samples_per_s=args.sur_steps * args.sur_batch / train_s,
        loss_first=float(log[0]), loss_last=float(log[-1]),
        tau=tau, target_mae=args.sur_mae, fallback_fraction=nfb / R, mae=mae,
        queries_per_s=q_per_s, speedup_vs_plain=q_per_s / plain_rays_per_s,
        network_only=dict(queries_per_s=R / mlp_s, mae=mae_net, ms=mlp_s * 1000.0,
                          tflops=MLP_FLOPS_PER_QUERY * R / mlp_s / 1e12,
                          mfma_frac=MLP_FLOPS_PER_QUERY * R / mlp_s / 1e12 / BF16_PEAK_TFLOPS),
        ms=fb_s * 1000.0,
    )


# FP32 operations per (Gaussian, direction) of the shading sum, counted from
# the formulas: direction in the normal frame and its normalisation 15, the
# two angles and the bilinear map lookup 30, the SH basis and its three dot
# products 39, the microfacet specular 45, the accumulation 9
SHADE_FLOPS = 138
FP32_PEAK_TFLOPS = 157.3


def shade_leg(torch, g, dirs, prm, vis_ray):
    """Per-Gaussian PBR colour (Eq. (10)) from the traced visibility, with
    seeded materials, environment map and camera."""
    from paper_2311_16043_amd import shade_pbr
    from workloads import materials
    n, K = vis_ray.shape
    m = materials.make_materials(n, 0)
    dev = vis_ray.device
    alb, rough, sh = (torch.from_numpy(m[k]).to(dev) for k in ("albedo", "roughness", "sh"))
    env = torch.from_numpy(materials.make_env(0)).to(dev)
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    shade_pbr(g, dirs, vis_ray, alb, rough, sh, env, materials.CAMERA, params=prm, out=out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        shade_pbr(g, dirs, vis_ray, alb, rough, sh, env, materials.CAMERA, params=prm, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    pairs = n * K
    tflops = SHADE_FLOPS * pairs / (ms / 1000.0) / 1e12
    hbm = (4 * pairs + n * 4 * (3 + 3 + 3 + 1 + 27 + 3)) / (ms / 1000.0) / 1e9
    return dict(pairs=pairs, ms=ms, pairs_per_s=pairs / (ms / 1000.0), mean_color=float(out.mean()),
                roofline={"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": tflops / FP32_PEAK_TFLOPS, "flops_per_pair": SHADE_FLOPS},
                hbm_gbs=hbm)


def retrace_leg(torch, g, prm, bvh, iters=20):
    """Training-time tracing (Sec. 3.3 and 5.1): every iteration draws a new
    turn of the 64 Fibonacci directions about each normal and re-traces all
    Gaussians (vis_ray and vis_mean), table upload included."""
    from paper_2311_16043_amd import trace_visibility
    from workloads import scenes
    rng = np.random.Generator(np.random.PCG64(16043 + 7))
    dev = g.mean.device
    K = 64
    vr = torch.empty((g.n, K), dtype=torch.float32, device=dev)
    vm = torch.empty((g.n,), dtype=torch.float32, device=dev)
    tables = [scenes.rotated_dirs(K, float(a)) for a in rng.uniform(0, 2 * np.pi, iters + 2)]
    trace_visibility(bvh, g, torch.from_numpy(tables[0]).to(dev), prm, out_ray=vr, out_mean=vm)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for it in range(iters):
        trace_visibility(bvh, g, torch.from_numpy(tables[it + 1]).to(dev), prm, out_ray=vr, out_mean=vm)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / iters
    return dict(directions=K, iterations=iters, ms_per_iteration=dt * 1000.0, rays_per_s=g.n * K / dt)


def edit_leg(torch, sc, g, dirs, prm):
    """Scene edit (Sec. 4.3): turn the sphere of the object scene by 0.5 rad
    about the vertical and shift it by (0.8, 0.3, 0); update the tree by refit
    (order and topology kept) or by a full rebuild, and trace both."""
    from paper_2311_16043_amd import Gaussians, build_bvh, refit_bvh, trace_visibility
    from workloads import scenes
    dev = g.mean.device
    sel = np.nonzero(sc["mean"][:, 2] > 0.05)[0]
    g2 = Gaussians.from_scene(scenes.rigid_move(sc, sel, 0.5, [0.8, 0.3, 0.0]), device=dev)
    bvh_r = build_bvh(g)
    L = __import__("paper_2311_16043_amd")._lib.load()
    ws = torch.empty(int(L.rv_build_workspace_bytes(g.n)), dtype=torch.uint8, device=dev)
    vr = torch.empty((g.n, int(dirs.shape[0])), dtype=torch.float32, device=dev)
    vm = torch.empty((g.n,), dtype=torch.float32, device=dev)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            r = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), r

    refit_ms, _ = timed(lambda: refit_bvh(bvh_r, g2, workspace=ws))
    build_ms, bvh_b = timed(lambda: build_bvh(g2, workspace=ws))
    trace_refit_ms, _ = timed(lambda: trace_visibility(bvh_r, g2, dirs, prm, out_ray=vr, out_mean=vm))
    trace_build_ms, _ = timed(lambda: trace_visibility(bvh_b, g2, dirs, prm, out_ray=vr, out_mean=vm))
    return dict(moved=int(sel.size), refit_ms=refit_ms, rebuild_ms=build_ms, trace_after_refit_ms=trace_refit_ms,
                trace_after_rebuild_ms=trace_build_ms)


def vis_sh_leg(torch, g, dirs, prm, bvh):
    """Visibility compressed to 9 SH coefficients per Gaussian, traced with no
    per-ray output (same rays as the step)."""
    from paper_2311_16043_amd import trace_visibility_sh
    n, K = g.n, int(dirs.shape[0])
    L = __import__("paper_2311_16043_amd")._lib.load()
    ws = torch.empty(int(L.rv_trace_sh_workspace_bytes(n, K)), dtype=torch.uint8, device=g.mean.device)
    trace_visibility_sh(bvh, g, dirs, prm, workspace=ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        trace_visibility_sh(bvh, g, dirs, prm, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    return dict(ms=ms, rays_per_s=n * K / (ms / 1000.0), output_bytes=n * 9 * 4, per_ray_output_bytes=n * K * 4,
                workspace_bytes=int(ws.numel()))


def adjoint_leg(torch, dev):
    """Forward and adjoint on the differentiation workload (200,000 Gaussians x
    128 hemisphere directions) with the loss L = mean_i (Vbar_i - y_i)^2: the
    upstream gradient is dL/dVbar_i = 2 (Vbar_i - y_i) / n. Times the adjoint
    with the forward's saved transmittances (one traversal per ray) and without
    (it re-traces to recover them)."""
    from paper_2311_16043_amd import Gaussians, TraceParams, build_bvh, trace_visibility, trace_visibility_backward
    from workloads import scenes
    sc = scenes.make_scene("diff")
    g = Gaussians.from_scene(sc, device=dev)
    dirs = torch.from_numpy(scenes.preset_dirs("diff")).to(dev)
    prm = TraceParams(dir_mode=scenes.PRESETS["diff"]["dir_mode"])
    bvh = build_bvh(g)
    y = torch.from_numpy(np.random.Generator(np.random.PCG64(16043 + 3)).uniform(0, 1, g.n).astype(np.float32)).to(dev)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            r = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), r

    fwd_ms, (vr, vm) = timed(lambda: trace_visibility(bvh, g, dirs, prm))
    gmean = 2.0 * (vm - y) / g.n
    bwd_ms, _ = timed(lambda: trace_visibility_backward(bvh, g, dirs, prm, grad_vis_mean=gmean, vis_ray_fwd=vr))
    bwd2_ms, _ = timed(lambda: trace_visibility_backward(bvh, g, dirs, prm, grad_vis_mean=gmean))
    rays = g.n * int(dirs.shape[0])
    return dict(workload="differentiation: 200,000 object-scale Gaussians x 128 hemisphere directions",
                rays=rays, forward_ms=fwd_ms, backward_ms=bwd_ms, backward_rays_per_s=rays / (bwd_ms / 1000.0),
                backward_retrace_ms=bwd2_ms, backward_over_forward=bwd_ms / fwd_ms)


def copy_probe(torch, nbytes=1 << 31, iters=5):
    """Achievable HBM bandwidth of the library's streaming copy: read + write bytes / time."""
    from paper_2311_16043_amd import stream_copy
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    stream_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        stream_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1000.0 / iters
    return dict(bytes_per_copy=nbytes, gbs=2 * nbytes / dt / 1e9, ms=dt * 1000.0)


def cpu_baseline(scene, dirs, dir_mode, target_s):
    """The FP64 oracle, as it stands, on a bounded seeded sample of the same rays."""
    import oracle
    from workloads import scenes
    n, K = scene["mean"].shape[0], dirs.shape[0]
    t = time.perf_counter()
    oracle.trace_rays(scene, dirs, dir_mode, scenes.sample_ray_ids(n, K, 1, seed=98))
    setup = time.perf_counter() - t
    pilot = scenes.sample_ray_ids(n, K, max(16, min(512, 512 * 300_000 // n)), seed=99)
    t = time.perf_counter()
    oracle.trace_rays(scene, dirs, dir_mode, pilot)
    per_ray = max(time.perf_counter() - t - setup, 1e-3) / pilot.size
    count = int(max(64, min(1 << 18, target_s / max(per_ray, 1e-9))))
    ids = scenes.sample_ray_ids(n, K, count, seed=100)
    t = time.perf_counter()
    oracle.trace_rays(scene, dirs, dir_mode, ids)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=count / dt, unit="rays/s", cores=cores, kind="oracle",
                sample=f"{count} seeded rays of the same workload, FP64 brute force over all {n} Gaussians "
                       f"(no BVH), {dt:.1f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path would shard by contiguous Morton ranges of origins, one range per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2311_16043_amd import Gaussians, TraceParams, build_bvh, trace_stats, trace_visibility
    from workloads import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_probe(torch)}), flush=True)
        return
    name = args.workload
    sc = scenes.make_scene(name)
    dirs_np = scenes.preset_dirs(name)
    dir_mode = scenes.PRESETS[name]["dir_mode"]
    prm = TraceParams(dir_mode=dir_mode)
    g = Gaussians.from_scene(sc, device=dev)
    dirs = torch.from_numpy(dirs_np).to(dev)
    n, K = g.n, int(dirs.shape[0])
    rays = n * K
    vis_ray = torch.empty((n, K), dtype=torch.float32, device=dev)
    vis_mean = torch.empty((n,), dtype=torch.float32, device=dev)
    L = __import__("paper_2311_16043_amd")._lib.load()
    ws = torch.empty(int(L.rv_build_workspace_bytes(n)), dtype=torch.uint8, device=dev)
    tws = torch.empty(int(L.rv_trace_workspace_bytes(n, K)), dtype=torch.uint8, device=dev)

    def step(ev=None):
        if ev:
            ev[0].record()
        bvh = build_bvh(g, workspace=ws)
        if ev:
            ev[1].record()
        trace_visibility(bvh, g, dirs, prm, out_ray=vis_ray, out_mean=vis_mean, workspace=tws)
        if ev:
            ev[2].record()
        return bvh

    for _ in range(args.warmup):
        bvh = step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done: n={n} K={K} rays={rays}", file=sys.stderr, flush=True)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        bvh = step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    build_ms = [e[0].elapsed_time(e[1]) for e in evs]
    trace_ms = [e[1].elapsed_time(e[2]) for e in evs]
    ms_per_step = 1000.0 * wall / args.steps
    value = rays * args.steps / wall

    # algorithmic bytes of the traversal kernel (deterministic for this BVH):
    # origin data, one compressed four-wide record per node visit, one leaf
    # record per leaf test, the ray's output, and the mean per Gaussian
    st = trace_stats(bvh, g, dirs, prm)
    alg_bytes = 24 * rays + NODE_BYTES * st["nodes"] + LEAF_BYTES * st["leaves"] + 4 * rays + 4 * n
    trace_s = float(np.mean(trace_ms)) / 1000.0
    achieved = alg_bytes / trace_s / 1e9
    print(f"[bench] step {ms_per_step:.2f} ms (build {np.mean(build_ms):.3f} ms, trace {np.mean(trace_ms):.3f} ms); "
          f"nodes/ray {st['nodes'] / rays:.2f} leaves/ray {st['leaves'] / rays:.2f} hits/ray {st['hits'] / rays:.2f}",
          file=sys.stderr, flush=True)

    out = {
        "metric": "visibility rays/sec (plain trace vs surrogate) at <=0.02 mean abs vis error",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": {"object": "object-scale: unit sphere on a 4x4 plane, 300,000 surface Gaussians x 256 "
                                   "hemisphere directions",
                         "multi": "multi-object: 8 objects x 150,000 surface Gaussians x 512 hemisphere directions",
                         "tiny": "tiny: 2,000 Gaussians x 64 sphere directions",
                         "surrogate": "surrogate-scale: 20 objects x 150,000 surface Gaussians x 1,024 hemisphere "
                                      "directions"}[name],
            "n_gaussians": n, "directions": K, "rays_per_step": rays,
            "step": "build_bvh + trace_visibility (vis_ray and vis_mean)",
        },
        "build_ms": float(np.mean(build_ms)),
        "trace_ms": float(np.mean(trace_ms)),
        "trace_rays_per_s": rays / trace_s,
        "roofline": {
            "kernel": "k_trace_stream",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic() if name == "object" else None,
            "alg_bytes_per_launch": alg_bytes,
            "nodes_per_ray": st["nodes"] / rays,
            "leaves_per_ray": st["leaves"] / rays,
            "hits_per_ray": st["hits"] / rays,
            # brute force reads every other Gaussian's record per ray
            "brute_force_bytes_per_ray": LEAF_BYTES * (n - 1),
            "work_avoided": LEAF_BYTES * (n - 1) * rays / alg_bytes,
        },
    }
    if not args.no_surrogate and name != "tiny":
        out["surrogate"] = surrogate_leg(args, torch, g, dirs, prm, bvh, vis_ray, rays / trace_s)
        print(f"[bench] surrogate: {json.dumps(out['surrogate'])}", file=sys.stderr, flush=True)
    if name == "object":
        out["edit"] = edit_leg(torch, sc, g, dirs, prm)
        print(f"[bench] edit: {json.dumps(out['edit'])}", file=sys.stderr, flush=True)
        out["retrace"] = retrace_leg(torch, g, prm, bvh)
        print(f"[bench] retrace: {json.dumps(out['retrace'])}", file=sys.stderr, flush=True)
    out["vis_sh"] = vis_sh_leg(torch, g, dirs, prm, bvh)
    print(f"[bench] vis_sh: {json.dumps(out['vis_sh'])}", file=sys.stderr, flush=True)
    if not args.no_shade:
        out["pbr"] = shade_leg(torch, g, dirs, prm, vis_ray)
        print(f"[bench] pbr: {json.dumps(out['pbr'])}", file=sys.stderr, flush=True)
    if not args.no_adjoint and name == "object":
        out["adjoint"] = adjoint_leg(torch, dev)
        print(f"[bench] adjoint: {json.dumps(out['adjoint'])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, dirs_np, dir_mode, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
