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
    V, U, _ = mlp.forward(theta, x, d, -2 * np.ones(3), 2 * np.ones(3))
    assert np.all((V > 0) & (V < 1)) and np.all(U >= 0)
