"""FP64 reference of the MLP visibility surrogate. TEST INFRASTRUCTURE ONLY.

The network (not part of the paper; it stands in for repeated tracing of the
visibility term V of Eq. (9)):

  input   x (3, mapped to [-1, 1] by the scene box) and unit direction d (3)
  encode  each scalar u -> [u, sin(2^l pi u), cos(2^l pi u)], l = 0, 1, 2;
          42 features, zero-padded to 64
  hidden  4 layers of 256 with ReLU (64->256, then 3 x 256->256)
  head    256 -> 2: V = sigmoid(z0), U = z1 (predicted |T - V|)
  loss    mean over the batch of BCE(V, T) + (U - |T - V|)^2, V held constant
          in the second term (no gradient flows from it into z0); the squared
          error makes U the conditional mean of |T - V|, the quantity whose
          largest values the tracer fallback should take. U is linear in z1:
          a saturating activation (softplus) let the head collapse to ~0
          where its gradient vanished, in short training runs
  Adam    Kingma & Ba (2015) with bias correction, cosine-decayed step size

Parameters are one flat FP64 vector in the order W1, b1, ..., W5, b5 with
W_l stored [in][out] row-major.

bf16=True rounds to bfloat16 (round to nearest even) exactly where the GPU
kernels feed their matrix cores: weights and layer inputs of every forward
product, and the pre-activation gradients entering the backward products;
everything else (accumulation, biases, nonlinearities, the loss) is FP64 here
and FP32 on the GPU.
"""
from __future__ import annotations

import math

import numpy as np

N_ENC = 42
N_IN = 64
HID = 256
N_OUT = 2
SHAPES = [(N_IN, HID), (HID, HID), (HID, HID), (HID, HID), (HID, N_OUT)]


def n_params() -> int:
    return sum(a * b + b for a, b in SHAPES)


def unpack(theta: np.ndarray):
    """[(W [in, out], b [out]), ...] views into the flat parameter vector."""
    out = []
    o = 0
    for a, b in SHAPES:
        W = theta[o:o + a * b].reshape(a, b)
        o += a * b
        bias = theta[o:o + b]
        o += b
        out.append((W, bias))
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via the binary32 value, as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def normalize(x: np.ndarray, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    span = hi - lo
    safe = np.where(span > 0, span, 1.0)
    return np.where(span > 0, 2.0 * (np.asarray(x, np.float64) - lo) / safe - 1.0, 0.0)


def encode(xn: np.ndarray, d: np.ndarray) -> np.ndarray:
    """[n, 64]: per scalar u of (xn, d): u, sin(pi u), cos(pi u), sin(2 pi u), cos(2 pi u),
    sin(4 pi u), cos(4 pi u); columns 42..63 are zero."""
    u = np.concatenate([np.asarray(xn, np.float64), np.asarray(d, np.float64)], axis=1)
    n = u.shape[0]
    out = np.zeros((n, N_IN))
    for a in range(6):
        out[:, 7 * a] = u[:, a]
        for lvl in range(3):
            w = (2.0 ** lvl) * math.pi
            out[:, 7 * a + 1 + 2 * lvl] = np.sin(w * u[:, a])
            out[:, 7 * a + 2 + 2 * lvl] = np.cos(w * u[:, a])
    return out


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(theta, x, d, lo, hi, bf16_emulation: bool = True):
    """(V [n], U [n], cache) for inputs x [n, 3], d [n, 3]."""
    r = bf16 if bf16_emulation else (lambda a: np.asarray(a, np.float64))
    layers = unpack(np.asarray(theta, np.float64))
    h = encode(normalize(x, lo, hi), d)
    hs, zs = [], []
    for li, (W, b) in enumerate(layers):
        hin = r(h)
        hs.append(hin)
        z = hin @ r(W) + b
        zs.append(z)
        h = np.maximum(z, 0.0) if li < len(layers) - 1 else z
    z = zs[-1]
    V = _sigmoid(z[:, 0])
    U = z[:, 1].copy()
    return V, U, dict(hs=hs, zs=zs, V=V, U=U)


def head_abs_terms(theta, cache):
    """[n, 2]: sum_k |W5[k, c] h4[k]| for each sample and head output c, the
    magnitudes of the terms of the last product (bf16 operands). One BF16
    rounding of a layer input that comes out differently moves an output by
    about 2^-8 of such a sum; it is the error scale of the outputs."""
    W5 = unpack(np.asarray(theta, np.float64))[-1][0]
    return np.abs(cache["hs"][-1]) @ np.abs(bf16(W5))


def loss_and_grad(theta, x, d, T, lo, hi, bf16_emulation: bool = True, e_fixed=None):
    """(mean loss, gradient [n_params]) of BCE(V, T) + (U - e)^2 with e = |T - V|
    held constant (stop-gradient). e_fixed replaces e by given values, so that
    finite differences of the returned loss see exactly the objective whose
    gradient is returned."""
    r = bf16 if bf16_emulation else (lambda a: np.asarray(a, np.float64))
    theta = np.asarray(theta, np.float64)
    T = np.asarray(T, np.float64)
    V, U, c = forward(theta, x, d, lo, hi, bf16_emulation)
    n = T.shape[0]
    eps = 1e-12
    e = np.abs(T - V) if e_fixed is None else np.asarray(e_fixed, np.float64)
    bce = -(T * np.log(np.maximum(V, eps)) + (1 - T) * np.log(np.maximum(1 - V, eps)))
    loss = float(np.mean(bce + (U - e) ** 2))
    z5 = c["zs"][-1]
    dz = np.zeros((n, N_OUT))
    dz[:, 0] = (V - T) / n
    dz[:, 1] = 2.0 * (U - e) / n
    layers = unpack(theta)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        dzr = r(dz)
        gW = c["hs"][li].T @ dzr
        gb = dz.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            dh = dzr @ r(W).T
            dz = dh * (c["zs"][li - 1] > 0)
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, flat


def lr_at(step: int, total: int, lr: float, lr_min: float) -> float:
    """Cosine decay from lr (step 0) to lr_min (step total)."""
    if total <= 0:
        return lr
    t = min(max(step, 0), total) / total
    return lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * t))


def adam_step(theta, m, v, g, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1) -> (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014; Vigna's constants)."""
    x = (x + 0x9E3779B97F4A7C15) & _M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & _M64
    return x ^ (x >> 31)


def batch_indices(seed: int, step: int, batch: int, n_samples: int) -> np.ndarray:
    """Training-sample indices of one step: splitmix64(seed ^ splitmix64(step * 2^32 + slot)) mod n."""
    return np.array([splitmix64(seed ^ splitmix64(((step << 32) + s) & _M64)) % n_samples for s in range(batch)],
                    dtype=np.int64)
