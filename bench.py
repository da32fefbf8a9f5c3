"""Benchmark: visibility rays/s of the plain BVH tracer against the MLP
surrogate with tracer fallback, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload surrogate]

Default workload: 20 objects of 150,000 surface Gaussians (3,000,000) on a
ground plane, 1,024 hemisphere directions each (3.07e9 rays), the multi-object
composition of the paper's relighting use (Sec. 4.3) traced for visibility
pre-computation (Sec. 4.2). A timed step is one pass of the plain path over
that input: LBVH build (bounds, Morton keys, radix sort, radix tree, refit)
then the traversal writing every ray's transmittance and each Gaussian's mean
visibility. Inputs are resident in HBM before timing starts.

The surrogate path is measured in the same run on the same workload: the MLP
is trained on 50M tracer samples, the fallback threshold is picked on
held-out queries for a mean absolute error <= 0.02 against the tracer, and
all 3.07e9 queries are answered by the network with the flagged ones traced.
`value` is the plain path's rate; the surrogate's queries/s, its error and
its fallback fraction sit beside it. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3

KERNEL_SOURCES = ["paper_2311_16043_amd/csrc/trace.hip", "paper_2311_16043_amd/csrc/trace_core.h",
                  "paper_2311_16043_amd/csrc/build.hip", "paper_2311_16043_amd/csrc/rv_internal.h"]

WORKLOADS = {
    "surrogate": "surrogate-scale composition: 20 objects x 150,000 surface Gaussians (3,000,000) x 1,024 "
                 "hemisphere directions",
    "multi": "multi-object composition: 8 objects x 150,000 surface Gaussians x 512 hemisphere directions",
    "object": "object-scale: unit sphere on a 4x4 plane, 300,000 surface Gaussians x 256 hemisphere directions",
    "tiny": "tiny: 2,000 Gaussians x 64 sphere directions",
}

NODE_BYTES = 48   # compressed four-wide node: origin, exponents and kinds, 24 plane bytes, 2 child indices
LEAF_BYTES = 48   # leaf record: mean, opacity, two whitening rows, s0 s1/s2, source index
RAY_BYTES = 24 + 4  # origin record and direction read, the ray's T written
MLP_FLOPS_PER_QUERY = 2 * (64 * 256 + 3 * 256 * 256 + 256 * 2)   # dense layers, padded input width 64


def sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# committed counter profiles of the traversal, per workload
TRAFFIC_PROFILES = {"object": "profiles/trace_object_scale_counters.md",
                    "surrogate": "profiles/trace_surrogate_counters.md"}


def recorded_traffic(workload: str):
    """HBM bytes per launch of k_trace_stream from the committed counter
    profile of this workload, if it was taken on the kernel sources as they
    are now (else None), with the file it came from."""
    path = TRAFFIC_PROFILES.get(workload, f"profiles/trace_{workload}_counters.md")
    try:
        text = open(os.path.join(ROOT, path)).read()
    except OSError:
        return None, path
    kv = {}
    for line in text.splitlines():
        if ": " in line:
            k, v = line.strip().split(": ", 1)
            kv[k.strip("- `")] = v.strip("` ")
    if kv.get("kernel_sources_sha256_16") != sources_hash():
        return None, path
    try:
        return float(kv["traffic_bytes_per_launch"]), path
    except (KeyError, ValueError):
        return None, path


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="surrogate", choices=list(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the all-core oracle baseline")
    ap.add_argument("--cpu1-seconds", type=float, default=5.0, help="target CPU time of the one-thread baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the streaming-copy probe (known-size reference for counters)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-shade", action="store_true", help="skip the PBR shading leg")
    ap.add_argument("--no-sh", action="store_true", help="skip the SH-compressed visibility leg")
    ap.add_argument("--sur-train-samples", type=int, default=50_000_000)
    ap.add_argument("--sur-steps", type=int, default=146496,
                    help="optimiser steps (146496 x 8192 = 24 passes over 50M; the fallback needed for MAE 0.02 "
                         "falls with the number of steps: at batches of 16384, 63 %% after two passes, 54 %% after "
                         "four, 50 %% after eight, 48 %% after 16, 47 %% after 24)")
    ap.add_argument("--sur-batch", type=int, default=8192)
    ap.add_argument("--sur-lr", type=float, default=2e-3, help="Adam step size, cosine-decayed to 1/40 of it")
    ap.add_argument("--sur-mae", type=float, default=0.02, help="target mean absolute visibility error")
    return ap.parse_args()


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_events(torch, fn, reps: int):
    """Median milliseconds of fn() over reps runs, HIP events on torch's
    current stream (the stream the library launches on), after one warm run."""
    fn()
    torch.cuda.synchronize()
    ts = []
    out = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), out


def surrogate_leg(args, torch, g, dirs, prm, bvh, vis_ray, plain_rays_per_s):
    """Train the MLP surrogate on the tracer's samples, pick the fallback
    threshold on held-out rays, then time the surrogate path over every query.
    The same threshold on the untrained network is the ablation."""
    from paper_2311_16043_amd import Surrogate, _lib, ray_setup
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
    untrained = Surrogate(lo, hi, seed=1, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    tlog = net.train(o, d, T_tr, steps=args.sur_steps, batch=args.sur_batch, lr=args.sur_lr, lr_min=args.sur_lr / 40,
                     seed=7)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    log(f"surrogate trained: {args.sur_steps} steps of {args.sur_batch} in {train_s:.2f} s, loss "
        f"{float(tlog[0]):.4f} -> {float(tlog[-1]):.4f}")
    del o, d, T_tr
    # threshold: rank held-out queries by predicted error, trace the top fraction
    oh, dh = ray_setup(g, dirs, ho_ids, prm)
    vh, uh = net.infer_xd(oh, dh)
    err = (vh - T_all[ho_ids]).abs()
    order = torch.argsort(uh, descending=True)
    e_sorted = err[order]
    kept_err = torch.flip(torch.cumsum(torch.flip(e_sorted, [0]), 0), [0]) / err.numel()  # MAE if the first j are traced
    # a 2.5 % margin so that the error over all queries stays within the
    # target (the standard error of the held-out estimate is ~0.5 % of it)
    ok = torch.nonzero(kept_err <= 0.975 * args.sur_mae)
    j = int(ok[0]) if ok.numel() else err.numel()
    tau = float(uh[order[j]]) if j < err.numel() else float("-inf")
    corr = float(torch.corrcoef(torch.stack([uh, err]))[0, 1])
    # timed: surrogate with fallback over all R queries, and the network alone
    out_v = torch.empty(R, dtype=torch.float32, device=dev)
    out_u = torch.empty(R, dtype=torch.float32, device=dev)
    ws = torch.empty(int(_lib.load().rv_surrogate_infer_workspace_bytes(R)), dtype=torch.uint8, device=dev)

    def sweep(m, tau_, with_bvh):
        box = {}

        def run():
            _, _, nfb = m.infer_grid(g, dirs, prm, 0, R, tau=tau_, bvh=bvh if with_bvh else None, out_vis=out_v,
                                     out_unc=out_u, workspace=ws)
            box["nfb"] = nfb
        ms, _ = timed_events(torch, run, 1)
        return ms / 1000.0, int(box["nfb"].item())

    mlp_s, _ = sweep(net, float("inf"), False)
    mae_net = float((out_v - T_all).abs().mean())
    fb_s, nfb = sweep(net, tau, True)
    mae = float((out_v - T_all).abs().mean())
    log(f"surrogate path: network {mlp_s * 1e3:.1f} ms, with fallback {fb_s * 1e3:.1f} ms "
        f"({nfb / R:.1%} traced), MAE {mae:.4f}")
    # ablation: the untrained network with the same threshold
    un_s, un_nfb = sweep(untrained, tau, True)
    un_mae = float((out_v - T_all).abs().mean())
    q_per_s = R / fb_s
    return dict(
        queries=R, train_samples=int(tr_ids.numel()), train_steps=args.sur_steps, batch=args.sur_batch,
        train_s=train_s, train_samples_per_s=args.sur_steps * args.sur_batch / train_s,
        loss_first=float(tlog[0]), loss_last=float(tlog[-1]),
        tau=tau, target_mae=args.sur_mae, fallback_fraction=nfb / R, mae=mae,
        corr_u_err_heldout=corr,
        queries_per_s=q_per_s, speedup_vs_plain=q_per_s / plain_rays_per_s, ms=fb_s * 1000.0,
        network_only=dict(queries_per_s=R / mlp_s, mae=mae_net, ms=mlp_s * 1000.0,
                          tflops=MLP_FLOPS_PER_QUERY * R / mlp_s / 1e12,
                          mfma_frac=MLP_FLOPS_PER_QUERY * R / mlp_s / 1e12 / BF16_PEAK_TFLOPS),
        untrained_same_tau=dict(fallback_fraction=un_nfb / R, mae=un_mae, ms=un_s * 1000.0,
                                queries_per_s=R / un_s),
    )


# FP32 operations per (Gaussian, direction) of the shading sum, counted from
# the formulas: direction in the normal frame and its normalisation 15, the
# two angles and the bilinear map lookup 30, the SH basis and its three dot
# products 39, the microfacet specular 45, the accumulation 9
SHADE_FLOPS = 138


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
    ms, _ = timed_events(torch, lambda: shade_pbr(g, dirs, vis_ray, alb, rough, sh, env, materials.CAMERA,
                                                  params=prm, out=out), 5)
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
    from paper_2311_16043_amd import Gaussians, _lib, build_bvh, refit_bvh, trace_visibility
    from workloads import scenes
    dev = g.mean.device
    sel = np.nonzero(sc["mean"][:, 2] > 0.05)[0]
    g2 = Gaussians.from_scene(scenes.rigid_move(sc, sel, 0.5, [0.8, 0.3, 0.0]), device=dev)
    bvh_r = build_bvh(g)
    ws = torch.empty(int(_lib.load().rv_build_workspace_bytes(g.n)), dtype=torch.uint8, device=dev)
    vr = torch.empty((g.n, int(dirs.shape[0])), dtype=torch.float32, device=dev)
    vm = torch.empty((g.n,), dtype=torch.float32, device=dev)
    refit_ms, _ = timed_events(torch, lambda: refit_bvh(bvh_r, g2, workspace=ws), 3)
    build_ms, bvh_b = timed_events(torch, lambda: build_bvh(g2, workspace=ws), 3)
    trace_refit_ms, _ = timed_events(torch, lambda: trace_visibility(bvh_r, g2, dirs, prm, out_ray=vr, out_mean=vm),
                                     3)
    trace_build_ms, _ = timed_events(torch, lambda: trace_visibility(bvh_b, g2, dirs, prm, out_ray=vr, out_mean=vm),
                                     3)
    return dict(moved=int(sel.size), refit_ms=refit_ms, rebuild_ms=build_ms, trace_after_refit_ms=trace_refit_ms,
                trace_after_rebuild_ms=trace_build_ms)


def vis_sh_leg(torch, g, dirs, prm, bvh, reps):
    """Visibility compressed to 9 SH coefficients per Gaussian, traced with no
    per-ray output (same rays as the step)."""
    from paper_2311_16043_amd import _lib, trace_visibility_sh
    n, K = g.n, int(dirs.shape[0])
    ws = torch.empty(int(_lib.load().rv_trace_sh_workspace_bytes(n, K)), dtype=torch.uint8, device=g.mean.device)
    ms, _ = timed_events(torch, lambda: trace_visibility_sh(bvh, g, dirs, prm, workspace=ws), reps)
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
    fwd_ms, (vr, vm) = timed_events(torch, lambda: trace_visibility(bvh, g, dirs, prm), 3)
    gmean = 2.0 * (vm - y) / g.n
    bwd_ms, _ = timed_events(torch, lambda: trace_visibility_backward(bvh, g, dirs, prm, grad_vis_mean=gmean,
                                                                      vis_ray_fwd=vr), 3)
    bwd2_ms, _ = timed_events(torch, lambda: trace_visibility_backward(bvh, g, dirs, prm, grad_vis_mean=gmean), 3)
    rays = g.n * int(dirs.shape[0])
    return dict(workload="differentiation: 200,000 object-scale Gaussians x 128 hemisphere directions",
                rays=rays, forward_ms=fwd_ms, backward_ms=bwd_ms, backward_rays_per_s=rays / (bwd_ms / 1000.0),
                backward_retrace_ms=bwd2_ms, backward_over_forward=bwd_ms / fwd_ms)


def copy_probe(torch, nbytes=1 << 31, iters=6):
    """Achievable HBM bandwidth of the library's streaming copy: read + write bytes / time."""
    from paper_2311_16043_amd import stream_copy
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    ms, _ = timed_events(torch, lambda: stream_copy(src, dst), iters)
    return dict(bytes_per_copy=nbytes, gbs=2 * nbytes / (ms / 1000.0) / 1e9, ms=ms)


def read_probe(torch, nbytes=1 << 31, iters=6):
    """Achievable HBM read bandwidth of the library's streaming read: bytes / time."""
    from paper_2311_16043_amd import stream_read
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    ms, _ = timed_events(torch, lambda: stream_read(src), iters)
    return dict(bytes=nbytes, gbs=nbytes / (ms / 1000.0) / 1e9, ms=ms)


def gather_probe_rate(torch, blocks: int, table_bytes=1 << 21, rounds=8192):
    """Achievable rate of the traversal's record reads: divergent 48-byte
    gathers (three 16-byte loads per lane) from an L2-resident table, with the
    traversal's resident blocks."""
    from paper_2311_16043_amd import gather_probe
    table = torch.randint(0, 1 << 30, (table_bytes // 4,), dtype=torch.int32, device="cuda:0")
    ms, _ = timed_events(torch, lambda: gather_probe(table, rounds, blocks), 3)
    nbytes = 48 * rounds * blocks * 256
    return dict(gbs=nbytes / (ms / 1000.0) / 1e9, ms=ms, table_bytes=table_bytes, blocks=blocks,
                records_per_thread=rounds)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(scene, dirs, dir_mode, target_s, target1_s):
    """The FP64 oracle, as it stands, on bounded seeded samples of the same
    rays: on every core the oracle's OpenMP loops use, and on one thread."""
    import oracle
    from workloads import scenes
    n, K = scene["mean"].shape[0], dirs.shape[0]
    threads = oracle.threads()

    def rate(count_target_s, seed):
        t = time.perf_counter()
        oracle.trace_rays(scene, dirs, dir_mode, scenes.sample_ray_ids(n, K, 1, seed=98))
        setup = time.perf_counter() - t
        # the oracle hands rays to its threads 16 at a time: a pilot of fewer
        # than 16 rays per thread leaves threads idle and overstates the cost
        pilot = scenes.sample_ray_ids(n, K, max(16 * oracle.threads(), min(512, 512 * 300_000 // n)), seed=99)
        t = time.perf_counter()
        oracle.trace_rays(scene, dirs, dir_mode, pilot)
        per_ray = max(time.perf_counter() - t - setup, 1e-3) / pilot.size
        count = int(max(16, min(1 << 18, count_target_s / max(per_ray, 1e-9))))
        ids = scenes.sample_ray_ids(n, K, count, seed=seed)
        t = time.perf_counter()
        oracle.trace_rays(scene, dirs, dir_mode, ids)
        return count, time.perf_counter() - t

    count, dt = rate(target_s, 100)
    oracle.set_threads(1)
    try:
        count1, dt1 = rate(target1_s, 101)
    finally:
        oracle.set_threads(threads)
    return dict(value=count / dt, unit="rays/s", cores=threads, kind="oracle",
                sample=f"{count} seeded rays of the same workload, FP64 brute force over all {n} Gaussians "
                       f"(no BVH), {dt:.1f} s on {threads} threads",
                one_thread=dict(value=count1 / dt1, unit="rays/s", sample=f"{count1} seeded rays, {dt1:.1f} s"),
                cpu_model=cpu_model())


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path would shard by contiguous Morton ranges of origins, one range per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2311_16043_amd import Gaussians, TraceParams, _lib, build_bvh, trace_stats, trace_visibility
    from workloads import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_probe(torch)}), flush=True)
        return
    name = args.workload
    log(f"workload {name}: generating the scene")
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
    L = _lib.load()
    ws = torch.empty(int(L.rv_build_workspace_bytes(n)), dtype=torch.uint8, device=dev)
    tws = torch.empty(256, dtype=torch.uint8, device=dev)   # queue counters (the rays go to vis_ray)

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
    log(f"warmup done: n={n} K={K} rays={rays}")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        bvh = step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    build_ms = [e[0].elapsed_time(e[1]) for e in evs]
    step_trace_ms = [e[1].elapsed_time(e[2]) for e in evs]
    ms_per_step = 1000.0 * wall / args.steps
    value = rays * args.steps / wall
    log(f"step {ms_per_step:.2f} ms (build {np.mean(build_ms):.3f} ms, trace with means "
        f"{np.mean(step_trace_ms):.3f} ms)")

    # the traversal kernel alone (queue clear + k_trace_stream, no row means),
    # HIP events on the stream it is launched on
    kernel_ms, _ = timed_events(torch, lambda: trace_visibility(bvh, g, dirs, prm, out_ray=vis_ray, want_mean=False,
                                                                workspace=tws), 2)
    # algorithmic bytes of the traversal (deterministic for this BVH up to a
    # few node visits): one compressed four-wide record per node visit, one
    # leaf record per leaf test, the ray's origin record and direction, its T
    st = trace_stats(bvh, g, dirs, prm)
    alg_bytes = RAY_BYTES * rays + NODE_BYTES * st["nodes"] + LEAF_BYTES * st["leaves"]
    kernel_s = kernel_ms / 1000.0
    achieved = alg_bytes / kernel_s / 1e9
    log(f"traversal kernel {kernel_ms:.2f} ms; nodes/ray {st['nodes'] / rays:.2f} leaves/ray "
        f"{st['leaves'] / rays:.2f} hits/ray {st['hits'] / rays:.2f}")
    blocks = int(torch.cuda.get_device_properties(0).multi_processor_count) * 6
    gp = gather_probe_rate(torch, blocks)
    cp = copy_probe(torch)
    rp = read_probe(torch)
    traffic, traffic_src = recorded_traffic(name)
    log(f"probes: record gather {gp['gbs']:.0f} GB/s, stream copy {cp['gbs']:.0f} GB/s, stream read "
        f"{rp['gbs']:.0f} GB/s")

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
            "workload": WORKLOADS[name],
            "n_gaussians": n, "directions": K, "rays_per_step": rays,
            "step": "build_bvh + trace_visibility (vis_ray and vis_mean); value is this plain path's rate",
        },
        "build_ms": float(np.mean(build_ms)),
        "trace_ms": float(np.mean(step_trace_ms)),
        "trace_kernel_ms": kernel_ms,
        "trace_rays_per_s": rays / kernel_s,
        "roofline": {
            "kernel": "k_trace_stream",
            # traversal reads its records through the per-CU vector-memory
            # path (TA/TD/L1) with divergent 16-byte lane loads, mostly served
            # by the L2; the peak is the measured rate of exactly that access
            # pattern (no published figure exists for it)
            "bound": "vmem",
            "achieved": achieved,
            "peak": gp["gbs"],
            "unit": "GB/s",
            "frac": achieved / gp["gbs"],
            "peak_source": "rv_gather_probe: divergent 48-byte record reads (three 16-byte loads per lane) from a "
                           "2 MiB L2-resident table, the traversal's resident blocks",
            "traffic": traffic,
            "traffic_source": (f"{traffic_src}: rocprofv3 FETCH_SIZE and WRITE_SIZE of k_trace_stream, calibrated "
                               f"by k_stream_copy; taken on these kernel sources") if traffic else
                              "no counter profile of these kernel sources",
            # counter-measured HBM bytes (98 % reads for this kernel) against
            # the achievable read bandwidth of the streaming read probe
            "hbm": ({"achieved": traffic / kernel_s / 1e9, "peak": rp["gbs"], "unit": "GB/s",
                     "frac": traffic / kernel_s / 1e9 / rp["gbs"],
                     "frac_of_copy": traffic / kernel_s / 1e9 / cp["gbs"],
                     "frac_of_spec": traffic / kernel_s / 1e9 / HBM_PEAK_GBS}
                    if traffic else None),
            "alg_bytes_per_launch": alg_bytes,
            "nodes_per_ray": st["nodes"] / rays,
            "leaves_per_ray": st["leaves"] / rays,
            "hits_per_ray": st["hits"] / rays,
            # brute force reads every other Gaussian's record per ray
            "brute_force_bytes_per_ray": LEAF_BYTES * (n - 1),
            "work_avoided": LEAF_BYTES * (n - 1) * rays / alg_bytes,
        },
        "probes": {"gather": gp, "copy": cp, "read": rp, "copy_frac_of_spec": cp["gbs"] / HBM_PEAK_GBS,
                   "read_frac_of_spec": rp["gbs"] / HBM_PEAK_GBS},
    }
    if not args.no_surrogate and name != "tiny":
        out["surrogate"] = surrogate_leg(args, torch, g, dirs, prm, bvh, vis_ray, rays / (np.mean(step_trace_ms) / 1e3))
        log(f"surrogate: {json.dumps(out['surrogate'])}")
    if name == "object":
        out["edit"] = edit_leg(torch, sc, g, dirs, prm)
        log(f"edit: {json.dumps(out['edit'])}")
        out["retrace"] = retrace_leg(torch, g, prm, bvh)
        log(f"retrace: {json.dumps(out['retrace'])}")
    if not args.no_sh:
        out["vis_sh"] = vis_sh_leg(torch, g, dirs, prm, bvh, 1 if rays > 1e9 else 3)
        log(f"vis_sh: {json.dumps(out['vis_sh'])}")
    if not args.no_shade:
        out["pbr"] = shade_leg(torch, g, dirs, prm, vis_ray)
        log(f"pbr: {json.dumps(out['pbr'])}")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(torch, dev)
        log(f"adjoint: {json.dumps(out['adjoint'])}")
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(sc, dirs_np, dir_mode, args.cpu_seconds, args.cpu1_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
