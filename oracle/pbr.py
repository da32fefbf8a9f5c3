"""FP64 reference of per-Gaussian physically based shading with pre-computed
visibility. TEST INFRASTRUCTURE ONLY: tests, smoke() and the CPU baseline of
bench.py use it; the library never does.

What is computed (Sec. 3.3, Eq. (7)-(10)): for Gaussian i with unit normal n,
albedo b, roughness r and indirect-light SH coefficients l, seen from the
direction w_o = normalize(camera - mu_i), the PBR colour is the sum over its
K sampled incident directions w_k (the tracer's directions, Sec. 3.3 and 4.2)

    c_i = sum_k (f_d + f_s(w_o, w_k)) L_i(w_k) max(w_k . n, 0) dw,
    L_i(w) = V_ik L_env(w) + sum_j l_j Y_j(w)          (Eq. (9)),
    f_d = b / pi,  f_s = D F G / (4 (n . w_k)(n . w_o))  (Eq. (8)),

with dw = 2 pi / K on the hemisphere (4 pi / K on the sphere). Readings of
what the paper leaves open (each is a choice, not the paper's statement):
  D   GGX / Trowbridge-Reitz with alpha = r^2 (Burley 2012);
  F   Schlick, F0 = f0 (0.04 for the dielectric the parameters describe);
  G   separable Smith with the GGX G1 of both directions;
  the 4 in f_s's denominator is the standard microfacet normalisation
      (the printed Eq. (8) omits it); h is the normalised half vector;
  f_s is 0 when the view lies below the surface (n . w_o <= 0);
  L_env  the 16 x 32 map is equirectangular in the world frame, +z up,
      row 0 at the +z pole, column 0 at azimuth -pi, texel centres at
      half-integer coordinates, sampled bilinearly (wrapping in azimuth,
      clamped at the poles) so that the colour is continuous in direction;
  Y_j the real spherical harmonics of degree <= 2 ("3-level SH"), in the
      order (0,0), (1,-1), (1,0), (1,1), (2,-2), (2,-1), (2,0), (2,1), (2,2).
"""
from __future__ import annotations

import math

import numpy as np

ENV_ROWS, ENV_COLS = 16, 32
N_SH = 9


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def onb(n):
    """Orthonormal (b1, b2) completing unit normals n [..., 3] (Duff et al., JCGT 2017)."""
    n = np.asarray(n, np.float64)
    sign = np.where(n[..., 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[..., 2])
    b = n[..., 0] * n[..., 1] * a
    b1 = np.stack([1.0 + sign * n[..., 0] ** 2 * a, sign * b, -sign * n[..., 0]], -1)
    b2 = np.stack([b, sign + n[..., 1] ** 2 * a, -n[..., 1]], -1)
    return b1, b2


def directions(normal, dirs, dir_mode: int):
    """Unit incident directions [n, K, 3] of every Gaussian: the table itself
    (dir_mode 0) or the table's local (x, y, z) rotated into the frame
    (b1, b2, n) of each normal (dir_mode 1), as the visibility rays use them."""
    dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
    normal = np.asarray(normal, np.float64).reshape(-1, 3)
    if dir_mode == 0:
        w = np.broadcast_to(dirs[None], (normal.shape[0],) + dirs.shape)
    else:
        n = _unit(normal)
        b1, b2 = onb(n)
        w = (dirs[None, :, 0:1] * b1[:, None] + dirs[None, :, 1:2] * b2[:, None] + dirs[None, :, 2:3] * n[:, None])
    return _unit(w)


def env_lookup(env, w):
    """Bilinear sample of the equirectangular map env [16, 32, C] in directions w [..., 3]."""
    env = np.asarray(env, np.float64)
    w = np.asarray(w, np.float64)
    theta = np.arctan2(np.hypot(w[..., 0], w[..., 1]), w[..., 2])       # [0, pi]
    phi = np.arctan2(w[..., 1], w[..., 0])                             # (-pi, pi]
    u = (phi + math.pi) / (2.0 * math.pi) * ENV_COLS - 0.5
    v = theta / math.pi * ENV_ROWS - 0.5
    c0 = np.floor(u)
    r0 = np.floor(v)
    fu = (u - c0)[..., None]
    fv = (v - r0)[..., None]
    c0 = c0.astype(np.int64)
    r0 = r0.astype(np.int64)
    ca, cb = c0 % ENV_COLS, (c0 + 1) % ENV_COLS
    ra, rb = np.clip(r0, 0, ENV_ROWS - 1), np.clip(r0 + 1, 0, ENV_ROWS - 1)
    top = (1.0 - fu) * env[ra, ca] + fu * env[ra, cb]
    bot = (1.0 - fu) * env[rb, ca] + fu * env[rb, cb]
    return (1.0 - fv) * top + fv * bot


def sh_basis(w):
    """Real spherical harmonics of degree <= 2 at unit directions w [..., 3] -> [..., 9]."""
    w = np.asarray(w, np.float64)
    x, y, z = w[..., 0], w[..., 1], w[..., 2]
    c0 = 0.5 * math.sqrt(1.0 / math.pi)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    c2 = 0.5 * math.sqrt(15.0 / math.pi)
    c20 = 0.25 * math.sqrt(5.0 / math.pi)
    c22 = 0.25 * math.sqrt(15.0 / math.pi)
    return np.stack([np.full_like(x, c0), c1 * y, c1 * z, c1 * x, c2 * x * y, c2 * y * z,
                     c20 * (3.0 * z * z - 1.0), c2 * x * z, c22 * (x * x - y * y)], -1)


def ggx_D(nh, alpha):
    """GGX normal distribution D(h) for cos(n, h) = nh and width alpha."""
    a2 = np.asarray(alpha, np.float64) ** 2
    t = np.asarray(nh, np.float64) ** 2 * (a2 - 1.0) + 1.0
    return a2 / (math.pi * t * t)


def smith_G1(nv, alpha):
    """Smith masking of the GGX distribution for cos(n, v) = nv > 0."""
    nv = np.asarray(nv, np.float64)
    a2 = np.asarray(alpha, np.float64) ** 2
    return 2.0 * nv / (nv + np.sqrt(a2 + (1.0 - a2) * nv * nv))


def schlick_F(vh, f0):
    """Schlick's Fresnel approximation for cos(v, h) = vh."""
    return f0 + (1.0 - f0) * (1.0 - np.asarray(vh, np.float64)) ** 5


def specular_cos(n, wo, wi, roughness, f0):
    """f_s(w_o, w_i) (n . w_i) = D F G / (4 (n . w_o)), 0 unless both cosines are positive."""
    ni = np.sum(n * wi, -1)
    no = np.sum(n * wo, -1)
    h = _unit(wi + wo)
    nh = np.maximum(np.sum(n * h, -1), 0.0)
    vh = np.maximum(np.sum(wo * h, -1), 0.0)
    alpha = np.asarray(roughness, np.float64) ** 2
    ok = (ni > 0.0) & (no > 0.0)
    ni_s, no_s = np.where(ok, ni, 1.0), np.where(ok, no, 1.0)
    val = ggx_D(nh, alpha) * schlick_F(vh, f0) * smith_G1(ni_s, alpha) * smith_G1(no_s, alpha) / (4.0 * no_s)
    return np.where(ok, val, 0.0)


def shade(mean, normal, dirs, dir_mode: int, vis, albedo, roughness, sh, env, camera, f0: float = 0.04):
    """(colour [n, 3], sum of |terms| [n, 3]) of Eq. (10) for every Gaussian; vis [n, K]."""
    mean = np.asarray(mean, np.float64).reshape(-1, 3)
    normal = np.asarray(normal, np.float64).reshape(-1, 3)
    vis = np.asarray(vis, np.float64).reshape(mean.shape[0], -1)
    K = vis.shape[1]
    n = _unit(normal)
    w = directions(n, dirs, dir_mode)                                       # [n, K, 3]
    wo = _unit(np.asarray(camera, np.float64)[None] - mean)                 # [n, 3]
    cos_i = np.maximum(np.sum(n[:, None] * w, -1), 0.0)                     # [n, K]
    spec = specular_cos(n[:, None], wo[:, None], w, np.asarray(roughness, np.float64)[:, None], f0)
    light = vis[..., None] * env_lookup(env, w) + np.einsum("nkj,njc->nkc", sh_basis(w),
                                                             np.asarray(sh, np.float64).reshape(-1, N_SH, 3))
    dw = (2.0 if dir_mode == 1 else 4.0) * math.pi / K
    diffuse = np.asarray(albedo, np.float64)[:, None, :] / math.pi * cos_i[..., None]
    terms = (diffuse + spec[..., None]) * light * dw
    return terms.sum(1), np.abs(terms).sum(1)
