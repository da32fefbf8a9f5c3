"""Pins of the surrogate-network oracle: bfloat16 rounding against torch's
conversion, the encoding at closed-form points, the analytic gradient against
FP64 central differences, Adam against its published update equations."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp
from workloads import mlp_init


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10 ** rng.uniform(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, -7.5e-39]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(x).astype(np.float32), ref)


def test_encoding_closed_form_points():
    xn = np.array([[0.0, 0.5, -1.0]])
    d = np.array([[1.0, 0.0, 0.25]])
    e = mlp.encode(xn, d)
    assert e.shape == (1, 64) and np.all(e[0, 42:] == 0)
    np.testing.assert_allclose(e[0, 0:7], [0, 0, 1, 0, 1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(e[0, 7:14], [0.5, 1, 0, 0, -1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(e[0, 14:21], [-1, 0, -1, 0, 1, 0, 1], atol=1e-15)
    s = math.sqrt(0.5)
    np.testing.assert_allclose(e[0, 35:42], [0.25, s, s, 1, 0, 0, -1], atol=1e-15)


def test_normalize_maps_box_to_unit_cube():
    lo, hi = np.array([-1.0, 2.0, 0.0]), np.array([3.0, 2.0, 5.0])
    x = np.array([[-1.0, 2.0, 0.0], [3.0, 2.0, 5.0], [1.0, 2.0, 2.5]])
    np.testing.assert_allclose(mlp.normalize(x, lo, hi), [[-1, 0, -1], [1, 0, 1], [0, 0, 0]])


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-2, 2, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    T = rng.uniform(0, 1, n)
    return x, d, T


def test_gradient_matches_central_differences_fp64():
    theta = mlp_init.he_uniform(3).astype(np.float64)
    theta += np.random.default_rng(1).normal(0, 0.05, theta.shape)  # nonzero biases
    x, d, T = _data(64, 2)
    lo, hi = np.array([-2.0, -2, -2]), np.array([2.0, 2, 2])
    V0, _, _ = mlp.forward(theta, x, d, lo, hi, bf16_emulation=False)
    e0 = np.abs(T - V0)   # the stop-gradient target, frozen for the differences
    _, g = mlp.loss_and_grad(theta, x, d, T, lo, hi, bf16_emulation=False)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(theta.size, 60, replace=False), np.arange(theta.size - 514, theta.size - 500)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grad(tp, x, d, T, lo, hi, bf16_emulation=False, e_fixed=e0)
        lm, _ = mlp.loss_and_grad(tm, x, d, T, lo, hi, bf16_emulation=False, e_fixed=e0)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_head_gradient_closed_form():
    """dL/dz0 of mean BCE with a sigmoid is (V - T)/n: check through b5[0]."""
    theta = mlp_init.he_uniform(4).astype(np.float64)
    x, d, T = _data(32, 3)
    lo, hi = -2 * np.ones(3), 2 * np.ones(3)
    V, U, _ = mlp.forward(theta, x, d, lo, hi)
    _, g = mlp.loss_and_grad(theta, x, d, T, lo, hi)
    assert abs(g[-2] - np.mean(V - T)) < 1e-12


def test_adam_matches_published_update():
    theta, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    g1, g2, lr = np.array([0.2]), np.array([-0.1]), 0.01
    t1, m1, v1 = mlp.adam_step(theta, m, v, g1, 1, lr)
    # step 1: m = 0.1 g, v = 0.001 g^2, bias-corrected to g and g^2
    assert abs(m1[0] - 0.02) < 1e-15 and abs(v1[0] - 0.001 * 0.04) < 1e-18
    assert abs(t1[0] - (0.5 - lr * 0.2 / (0.2 + 1e-8))) < 1e-15
    t2, m2, v2 = mlp.adam_step(t1, m1, v1, g2, 2, lr)
    m_ref = 0.9 * 0.02 + 0.1 * (-0.1)
    v_ref = 0.999 * 0.00004 + 0.001 * 0.01
    mh, vh = m_ref / (1 - 0.81), v_ref / (1 - 0.999 ** 2)
    assert abs(t2[0] - (t1[0] - lr * mh / (math.sqrt(vh) + 1e-8))) < 1e-15


def test_cosine_schedule_endpoints():
    assert mlp.lr_at(0, 100, 1e-3, 1e-5) == pytest.approx(1e-3)
    assert mlp.lr_at(100, 100, 1e-3, 1e-5) == pytest.approx(1e-5)
    assert mlp.lr_at(50, 100, 1e-3, 1e-5) == pytest.approx(0.5 * (1e-3 + 1e-5))


def test_forward_ranges_and_init_shapes():
    theta = mlp_init.he_uniform(7)
    assert theta.size == mlp.n_params() == 214530
    x, d, T = _data(100, 4)
    V, U, c = mlp.forward(theta, x, d, -2 * np.ones(3), 2 * np.ones(3))
    # V is a probability; U is the head's second output itself (linear)
    assert np.all((V > 0) & (V < 1)) and np.array_equal(U, c["zs"][-1][:, 1])


# Error scales of a BF16/FP32 evaluation: the network run with binary32
# accumulation (numpy float32 products and sums) and BF16 rounding of every
# product operand at the points the oracle rounds, against the FP64 oracle.
# The GPU parity tests apply the same bounds with the same constants.
# Outputs: one BF16 rounding of a layer input that comes out differently
# moves an output by about 2^-8 of the magnitude sum of the last product's
# terms, so each output is checked on its own. Gradients: a hidden
# pre-activation within rounding of zero switches its ReLU and adds or drops
# a whole term (94 % of samples have a unit within 2^-11 of its terms'
# magnitude sum of zero), so element bounds are either unsound or far above
# the gradient itself; each layer is checked by its relative Frobenius error
# and its largest element error relative to its largest element (one element
# off by a typical magnitude in a 64 x 256 layer moves the first to ~8e-3).
C_OUT = 1.0          # outputs: |dz_c| <= C_OUT 2^-8 sum_k |W5[k, c] h4[k]|
OUT_FROB = 1e-3      # relative Frobenius error of V and U
GRAD_FROB = 4e-3     # per-layer relative Frobenius error of W and b gradients
GRAD_MAXABS = 1e-2   # per-layer max |dg| / max |g|


def _f32_network(theta, x, d, T, lo, hi):
    """(z5 [n, 2], flat gradient) in binary32 with BF16 product operands."""
    bf = lambda a: mlp.bf16(a).astype(np.float32)
    layers = mlp.unpack(np.asarray(theta, np.float64))
    h = mlp.encode(mlp.normalize(x, lo, hi), d).astype(np.float32)
    hs, zs = [], []
    for li, (W, b) in enumerate(layers):
        hin = bf(h)
        hs.append(hin)
        z = (hin @ bf(W) + b.astype(np.float32)).astype(np.float32)
        zs.append(z)
        h = np.maximum(z, np.float32(0)) if li < len(layers) - 1 else z
    z5 = zs[-1]
    n = x.shape[0]
    V = (1 / (1 + np.exp(-z5[:, 0]))).astype(np.float32)
    U = z5[:, 1]
    e = np.abs(T.astype(np.float32) - V)
    dz = np.zeros((n, 2), np.float32)
    dz[:, 0] = (V - T) / np.float32(n)
    dz[:, 1] = np.float32(2) * (U - e) / np.float32(n)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        dzr = bf(dz)
        grads[li] = ((hs[li].T @ dzr).astype(np.float32), dz.sum(0, dtype=np.float32))
        if li > 0:
            dz = ((dzr @ bf(layers[li][0]).T) * (zs[li - 1] > 0)).astype(np.float32)
    return z5, np.concatenate([np.concatenate([a.reshape(-1), b]) for a, b in grads])


def layer_errors(got, ref):
    """[(name, relative Frobenius error, max |error| / max |ref|)] per W and b."""
    out, o = [], 0
    for li, (a, b) in enumerate(mlp.SHAPES):
        for name, size in (("W", a * b), ("b", b)):
            g, r = np.asarray(got[o:o + size], np.float64), ref[o:o + size]
            out.append((f"{name}{li + 1}", float(np.linalg.norm(g - r) / np.linalg.norm(r)),
                        float(np.abs(g - r).max() / np.abs(r).max())))
            o += size
    return out


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_binary32_network_within_the_output_and_gradient_bounds(seed):
    x, d, T = _data(2048, seed)
    theta = mlp_init.he_uniform(10 + seed)
    lo, hi = np.float32([-2, -2, -0.1]), np.float32([2, 2, 2.1])
    V, U, cache = mlp.forward(theta, x, d, lo, hi)
    A = mlp.head_abs_terms(theta, cache)
    _, g = mlp.loss_and_grad(theta, x, d, T, lo, hi)
    z5, g32 = _f32_network(theta, x, d, T, lo, hi)
    dz = np.abs(z5.astype(np.float64) - cache["zs"][-1])
    r_out = dz / (C_OUT * 2.0 ** -8 * A)
    V32 = 1 / (1 + np.exp(-z5[:, 0].astype(np.float64)))
    fv = np.linalg.norm(V32 - V) / np.linalg.norm(V)
    errs = layer_errors(g32, g)
    print(f"[bf16 bounds seed {seed}] outputs max |dz|/bound {r_out.max():.3f} (samples with any deviation "
          f"{(dz.max(1) > 1e-6 * A.max(1)).mean():.3f}), V Frobenius {fv:.1e}; gradients worst Frobenius "
          f"{max(e[1] for e in errs):.1e}, worst max-abs {max(e[2] for e in errs):.1e}", flush=True)
    assert np.all(r_out <= 1.0) and fv <= OUT_FROB
    assert all(f <= GRAD_FROB and m <= GRAD_MAXABS for _, f, m in errs), errs
    # the output bound is of the right size: the largest deviations reach a
    # visible fraction of it
    assert r_out.max() > 0.01
