"""MLP surrogate on the matrix cores vs the FP64 oracle with bfloat16 emulation
(relative Frobenius error <= 1e-2), grid inference with tracer fallback, and
what training on tracer samples gains over the untrained network."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2311_16043_amd import Gaussians, Surrogate, TraceParams, build_bvh, ray_setup, trace_rays, trace_visibility
from workloads import mlp_init, scenes

pytestmark = pytest.mark.gpu

BOX_LO, BOX_HI = np.array([-2.0, -2.0, -0.1]), np.array([2.0, 2.0, 2.1])


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(BOX_LO, BOX_HI, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    T = rng.uniform(0, 1, n) ** 2
    return x.astype(np.float32), d.astype(np.float32), T.astype(np.float32)


def _relf(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def _net(seed=11):
    w = mlp_init.he_uniform(seed)
    return Surrogate(BOX_LO, BOX_HI, init_weights=torch.from_numpy(w)), w


@pytest.mark.parametrize("n", [4096, 1000])
def test_forward_matches_oracle(n):
    net, w = _net()
    x, d, _ = _inputs(n, 1)
    vis, unc = net.infer_xd(torch.from_numpy(x), torch.from_numpy(d))
    torch.cuda.synchronize()
    V, U, _ = mlp.forward(w, x, d, BOX_LO.astype(np.float32), BOX_HI.astype(np.float32))
    ev, eu = _relf(vis.cpu().numpy(), V), _relf(unc.cpu().numpy(), U)
    print(f"[surrogate fwd n={n}] rel Frobenius V {ev:.2e} U {eu:.2e}; max |dV| "
          f"{np.abs(vis.cpu().numpy() - V).max():.2e}", flush=True)
    assert ev <= 1e-2 and eu <= 1e-2
    # the master copy holds the uploaded weights exactly
    assert np.array_equal(net.master.cpu().numpy(), w)


@pytest.mark.parametrize("n", [2048, 2000])
def test_loss_and_gradient_match_oracle(n):
    net, w = _net(12)
    x, d, T = _inputs(n, 2)
    loss, grad = net.loss_grad(torch.from_numpy(x), torch.from_numpy(d), torch.from_numpy(T))
    torch.cuda.synchronize()
    lref, gref = mlp.loss_and_grad(w, x, d, T, BOX_LO.astype(np.float32), BOX_HI.astype(np.float32))
    g = grad.cpu().numpy()
    assert abs(float(loss) - lref) <= 1e-3 * abs(lref)
    o = 0
    for li, (a, b) in enumerate(mlp.SHAPES):
        for name, size in (("W", a * b), ("b", b)):
            e = _relf(g[o:o + size], gref[o:o + size])
            print(f"[surrogate grad n={n}] layer {li + 1} {name}: rel Frobenius {e:.2e}", flush=True)
            assert e <= 1e-2, (li, name, e)
            o += size
    # deterministic
    _, grad2 = net.loss_grad(torch.from_numpy(x), torch.from_numpy(d), torch.from_numpy(T))
    assert torch.equal(grad, grad2)


def test_adam_step_matches_oracle():
    """One Adam step on a counter-hashed batch (the hash is implemented on both
    sides from the SplitMix64 definition). The moments are linear and quadratic
    in the gradient and are compared with the oracle's; the first update is
    ~lr sign(g) and may differ only where |g| is at the gradient's noise level;
    the weights must equal Adam's update applied to the kernel's own moments."""
    net, w = _net(13)
    x, d, T = _inputs(5000, 3)
    batch, lr, seed = 256, 1e-3, 77
    net.train(torch.from_numpy(x), torch.from_numpy(d), torch.from_numpy(T), steps=1, batch=batch, lr=lr,
              lr_min=lr, seed=seed, total_steps=10)
    torch.cuda.synchronize()
    got = net.master.cpu().numpy().astype(np.float64)
    gm, gv = net.adam_m.cpu().numpy().astype(np.float64), net.adam_v.cpu().numpy().astype(np.float64)
    idx = mlp.batch_indices(seed, 0, batch, 5000)
    _, g = mlp.loss_and_grad(w, x[idx], d[idx], T[idx], BOX_LO.astype(np.float32), BOX_HI.astype(np.float32))
    theta, m, v = mlp.adam_step(w.astype(np.float64), np.zeros(w.size), np.zeros(w.size), g, 1, lr)
    em, ev = _relf(gm, m), _relf(gv, v)
    # the kernel's weights follow from its own moments by the published update
    own = w - lr * (gm / 0.1) / (np.sqrt(gv / 0.001) + 1e-8)
    eo = np.max(np.abs(got - own)) / lr
    off = np.abs((got - w) - (theta - w)) > 0.1 * lr
    rms = np.sqrt(np.mean(g ** 2))
    print(f"[surrogate adam] rel Frobenius m {em:.2e} v {ev:.2e}; own-update max dev {eo:.2e} lr; "
          f"{off.mean():.2e} of weights off by > 0.1 lr, max |g|/RMS among them "
          f"{(np.abs(g[off]).max() / rms) if off.any() else 0:.2e}", flush=True)
    assert em <= 1e-2 and ev <= 1e-2
    assert eo <= 1e-3
    assert not off.any() or np.abs(g[off]).max() <= 0.1 * rms


def test_grid_inference_with_fallback_matches_tracer():
    sc = scenes.make_object_scene(20_000, 1)
    dirs = scenes.fibonacci_dirs(32, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    net = Surrogate(sc["mean"].min(0), sc["mean"].max(0), seed=5)
    prm = TraceParams()
    q0, qn = 1234, 100_001
    vis0, unc0, _ = net.infer_grid(g, dirs, prm, q0, qn)
    tau = float(unc0.median())
    vis, unc, nfb = net.infer_grid(g, dirs, prm, q0, qn, tau=tau, bvh=bvh)
    torch.cuda.synchronize()
    fb = (unc > tau).cpu().numpy()
    assert int(nfb.item()) == int(fb.sum()) and 0.3 < fb.mean() < 0.7
    assert torch.equal(unc, unc0)
    ids = np.arange(q0, q0 + qn, dtype=np.int64)
    traced = trace_rays(bvh, g, dirs, ids[fb], prm).cpu().numpy()
    v = vis.cpu().numpy()
    assert np.array_equal(v[fb].view(np.uint32), traced.view(np.uint32))
    assert np.array_equal(v[~fb].view(np.uint32), vis0.cpu().numpy()[~fb].view(np.uint32))
    # the grid queries see the tracer's own origins and directions
    o, dd = ray_setup(g, dirs, ids[:4096], prm)
    vx, _ = net.infer_xd(o, dd)
    assert np.array_equal(vx.cpu().numpy().view(np.uint32), vis0.cpu().numpy()[:4096].view(np.uint32))


def test_training_on_tracer_samples_beats_untrained_network():
    """Train on the tracer's own visibility: on held-out queries the trained
    network's error is far below the untrained one's, and its predicted error
    ranks the queries: the 20 % it flags for fallback carry well above the
    mean error of the rest, so tracing them lowers the combined error more
    than tracing a random 20 % would."""
    sc = scenes.make_object_scene(50_000, 1)
    K = 64
    dirs = scenes.fibonacci_dirs(K, True)
    g = Gaussians.from_scene(sc)
    bvh = build_bvh(g)
    vr, _ = trace_visibility(bvh, g, dirs, TraceParams())
    T_all = vr.reshape(-1)
    rng = np.random.default_rng(9)
    perm = rng.permutation(50_000 * K)
    train_ids, test_ids = perm[:2_000_000], perm[-200_000:]
    o, d = ray_setup(g, dirs, train_ids)
    net = Surrogate(sc["mean"].min(0), sc["mean"].max(0), seed=3)
    ot, dt = ray_setup(g, dirs, test_ids)
    v0, _ = net.infer_xd(ot, dt)
    Tt = T_all[torch.from_numpy(test_ids).cuda()]
    mae0 = float((v0 - Tt).abs().mean())
    log = net.train(o, d, T_all[torch.from_numpy(train_ids).cuda()], steps=600, batch=8192, lr=2e-3, lr_min=1e-4,
                    seed=1)
    v1, u1 = net.infer_xd(ot, dt)
    err = (v1 - Tt).abs()
    mae1 = float(err.mean())
    # fallback: queries with the largest predicted error are traced exactly
    tau = float(torch.quantile(u1, 0.8))
    fb = u1 > tau
    mae_fb = float(torch.where(fb, torch.zeros_like(err), err).mean())
    corr = float(torch.corrcoef(torch.stack([u1, err]))[0, 1])
    print(f"[surrogate train] loss {float(log[0]):.4f} -> {float(log[-1]):.4f}; MAE untrained {mae0:.4f}, "
          f"trained {mae1:.4f}, with {float(fb.float().mean()):.0%} fallback {mae_fb:.4f}; "
          f"corr(U, |err|) {corr:.2f}", flush=True)
    ratio = float(err[fb].mean() / err[~fb].mean())
    print(f"[surrogate train] mean |err| flagged / rest = {ratio:.2f}", flush=True)
    assert float(log[-1]) < float(log[0])
    assert mae1 < 0.5 * mae0
    assert ratio > 1.2 and mae_fb < 0.8 * mae1
