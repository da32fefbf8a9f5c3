"""Seeded synthetic Gaussian clouds and direction tables.

This module only draws inputs. It holds none of the visibility method's
arithmetic (no whitening, no ray construction, no tracing, no tree build), so
both the FP64 oracle and the HIP path can consume what it produces without
sharing any computation.

Every scene is a dict of C-contiguous float32 arrays:

  mean       [N, 3]   Gaussian centres
  quat       [N, 4]   rotation quaternions, (w, x, y, z) order, unit length
  log_scale  [N, 3]   natural-log standard deviations along the rotated axes
  opacity    [N]      opacity in (0, 1)
  normal     [N, 3]   unit surface normal (frame of the hemisphere directions)

The Gaussian parameterisation (centre, unit quaternion, scale vector, opacity)
and the per-Gaussian normal follow the paper's scene representation
(Sec. 3.1 and the extended per-Gaussian attribute list at the end of Sec. 3.3).

Shapes mirror the paper's workloads: single objects captured on a ground plane
(the object-scale scenes of its experiments) and multi-object compositions
(Sec. 4.3). The paper's datasets are not available; these procedural clouds
stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 16043

# Workload presets. Sizes only: the generators below draw the values.
PRESETS = {
    # uniform cube cloud, world-frame sphere directions
    "tiny": dict(kind="cube", n=2000, K=64, dir_mode=0),
    # unit sphere resting on a 4x4 plane
    "object": dict(kind="object", n=300_000, K=256, dir_mode=1),
    # 8 objects x 150k (object 0 is the ground plane)
    "multi": dict(kind="multi", n_objects=8, per_object=150_000, K=512, dir_mode=1),
    # 200k Gaussians from the object-scale generator, 128 directions
    "diff": dict(kind="object", n=200_000, K=128, dir_mode=1),
    # 20 objects x 150k, 1024 directions
    "surrogate": dict(kind="multi", n_objects=20, per_object=150_000, K=1024, dir_mode=1),
}
PRESET_INDEX = {"tiny": 0, "object": 1, "multi": 2, "diff": 3, "surrogate": 4}


def rng_for(name_or_index, extra: int = 0) -> np.random.Generator:
    idx = PRESET_INDEX[name_or_index] if isinstance(name_or_index, str) else int(name_or_index)
    return np.random.Generator(np.random.PCG64(SEED_BASE + idx + 1000 * extra))


# ----------------------------------------------------------------------------
# direction tables (Sec. 3.3: Fibonacci sampling of N_s directions)
# ----------------------------------------------------------------------------

def fibonacci_dirs(K: int, hemisphere: bool) -> np.ndarray:
    """Fibonacci (golden-angle) point set on the unit sphere or upper hemisphere.

    Point k has height z_k = 1 - (2k+1)/K on the sphere or 1 - (k+1/2)/K on the
    hemisphere (equal-area bands) and azimuth k * pi * (3 - sqrt(5)). Computed in
    float64, returned as float32 [K, 3]; the hemisphere points are in a local frame
    whose +z is the surface normal.
    """
    if K <= 0:
        return np.zeros((0, 3), np.float32)
    k = np.arange(K, dtype=np.float64)
    if hemisphere:
        z = 1.0 - (k + 0.5) / K
    else:
        z = 1.0 - (2.0 * k + 1.0) / K
    phi = k * (math.pi * (3.0 - math.sqrt(5.0)))
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    out = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    return np.ascontiguousarray(out.astype(np.float32))


# ----------------------------------------------------------------------------
# helpers for drawing oriented surface Gaussians
# ----------------------------------------------------------------------------

def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _quat_from_frames(R: np.ndarray) -> np.ndarray:
    """(w,x,y,z) unit quaternions of proper rotation matrices R[N,3,3] (Shepperd)."""
    m = R
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    cand = np.stack([tr, m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]], axis=1)
    sel = np.argmax(cand, axis=1)
    q = np.empty((R.shape[0], 4))
    # case 0: w largest
    s = np.sqrt(np.maximum(1.0 + tr, 1e-300)) * 2.0
    c0 = np.stack([0.25 * s, (m[:, 2, 1] - m[:, 1, 2]) / s,
                   (m[:, 0, 2] - m[:, 2, 0]) / s, (m[:, 1, 0] - m[:, 0, 1]) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m[:, 0, 0] - m[:, 1, 1] - m[:, 2, 2], 1e-300)) * 2.0
    c1 = np.stack([(m[:, 2, 1] - m[:, 1, 2]) / s, 0.25 * s,
                   (m[:, 0, 1] + m[:, 1, 0]) / s, (m[:, 0, 2] + m[:, 2, 0]) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m[:, 1, 1] - m[:, 0, 0] - m[:, 2, 2], 1e-300)) * 2.0
    c2 = np.stack([(m[:, 0, 2] - m[:, 2, 0]) / s, (m[:, 0, 1] + m[:, 1, 0]) / s,
                   0.25 * s, (m[:, 1, 2] + m[:, 2, 1]) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m[:, 2, 2] - m[:, 0, 0] - m[:, 1, 1], 1e-300)) * 2.0
    c3 = np.stack([(m[:, 1, 0] - m[:, 0, 1]) / s, (m[:, 0, 2] + m[:, 2, 0]) / s,
                   (m[:, 1, 2] + m[:, 2, 1]) / s, 0.25 * s], 1)
    for case, c in enumerate((c0, c1, c2, c3)):
        q[sel == case] = c[sel == case]
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return _unit(q)


def _surface_gaussians(rng: np.random.Generator, points: np.ndarray, normals: np.ndarray,
                       jitter: float = 0.01, normal_scale: float = 0.002,
                       tangent_range=(0.005, 0.02)) -> dict:
    """Gaussians flattened along the surface normal, as in the object-scale scenes."""
    n = points.shape[0]
    nrm = _unit(normals)
    helper = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    t1 = _unit(np.cross(nrm, helper))
    t2 = np.cross(nrm, t1)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=(n, 1))
    a1 = np.cos(ang) * t1 + np.sin(ang) * t2
    a2 = np.cross(nrm, a1)
    R = np.stack([a1, a2, nrm], axis=2)  # columns = principal axes
    quat = _quat_from_frames(R)
    lo, hi = math.log(tangent_range[0]), math.log(tangent_range[1])
    ls = np.empty((n, 3))
    ls[:, 0] = rng.uniform(lo, hi, n)
    ls[:, 1] = rng.uniform(lo, hi, n)
    ls[:, 2] = math.log(normal_scale)
    mean = points + rng.normal(0.0, jitter, size=(n, 3))
    opac = rng.beta(5.0, 1.0, size=n)
    opac = np.clip(opac, 1e-6, 1.0 - 1e-7)
    return dict(mean=mean, quat=quat, log_scale=ls, opacity=opac, normal=nrm)


def _finish(d: dict) -> dict:
    return {k: np.ascontiguousarray(np.asarray(v, dtype=np.float32)) for k, v in d.items()}


def _concat(parts) -> dict:
    return {k: np.concatenate([p[k] for p in parts], axis=0) for k in parts[0]}


# ----------------------------------------------------------------------------
# surface samplers (uniform by area)
# ----------------------------------------------------------------------------

def _sample_sphere(rng, n, centre, radius):
    v = _unit(rng.normal(size=(n, 3)))
    return np.asarray(centre)[None, :] + radius * v, v


def _sample_plane(rng, n, x0, x1, y0, y1, z=0.0):
    p = np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n), np.full(n, z)], 1)
    nrm = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    return p, nrm


def _sample_box(rng, n, half):
    """Axis-aligned box of half extents `half`, centred at origin, area-weighted faces."""
    hx, hy, hz = half
    areas = np.array([hy * hz, hy * hz, hx * hz, hx * hz, hx * hy, hx * hy])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    u = rng.uniform(-1.0, 1.0, n)
    v = rng.uniform(-1.0, 1.0, n)
    p = np.empty((n, 3))
    nrm = np.zeros((n, 3))
    for f in range(6):
        m = face == f
        ax = f // 2
        sgn = 1.0 if f % 2 == 0 else -1.0
        o1, o2 = [a for a in range(3) if a != ax]
        p[m, ax] = sgn * half[ax]
        p[m, o1] = u[m] * half[o1]
        p[m, o2] = v[m] * half[o2]
        nrm[m, ax] = sgn
    return p, nrm


def _sample_torus(rng, n, R, r):
    """Torus about +z (major radius R, minor r), uniform by area via rejection."""
    pts = []
    nrms = []
    got = 0
    while got < n:
        m = 2 * (n - got) + 64
        th = rng.uniform(0, 2 * math.pi, m)
        ph = rng.uniform(0, 2 * math.pi, m)
        keep = rng.uniform(0, 1, m) < (R + r * np.cos(ph)) / (R + r)
        th, ph = th[keep], ph[keep]
        nn = np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], 1)
        c = np.stack([R * np.cos(th), R * np.sin(th), np.zeros_like(th)], 1)
        pts.append(c + r * nn)
        nrms.append(nn)
        got += th.shape[0]
    return np.concatenate(pts)[:n], np.concatenate(nrms)[:n]


# ----------------------------------------------------------------------------
# scene generators
# ----------------------------------------------------------------------------

def make_cube_cloud(n: int = 2000, seed_index: int = 0) -> dict:
    """Uniform cloud: means U[-1,1]^3, log-scales U[ln .01, ln .05] per axis,
    uniformly random unit quaternions, opacity U[0.05, 0.99]."""
    rng = rng_for(seed_index)
    mean = rng.uniform(-1.0, 1.0, size=(n, 3))
    ls = rng.uniform(math.log(0.01), math.log(0.05), size=(n, 3))
    quat = _unit(rng.normal(size=(n, 4)))
    opac = rng.uniform(0.05, 0.99, size=n)
    normal = _unit(rng.normal(size=(n, 3)))
    return _finish(dict(mean=mean, quat=quat, log_scale=ls, opacity=opac, normal=normal))


def make_object_scene(n: int = 300_000, seed_index: int = 1) -> dict:
    """Unit sphere centred at (0,0,1) resting on the plane z=0 over [-2,2]^2.

    Points are split between sphere and plane by area; each becomes a Gaussian
    flattened along the surface normal (normal-axis scale 0.002, tangent scales
    log-uniform in [0.005, 0.02]), jittered by N(0, 0.01^2 I), opacity Beta(5,1).
    """
    rng = rng_for(seed_index)
    a_sph, a_pl = 4.0 * math.pi, 16.0
    n_sph = int(rng.binomial(n, a_sph / (a_sph + a_pl)))
    p1, n1 = _sample_sphere(rng, n_sph, (0.0, 0.0, 1.0), 1.0)
    p2, n2 = _sample_plane(rng, n - n_sph, -2.0, 2.0, -2.0, 2.0)
    pts = np.concatenate([p1, p2])
    nrm = np.concatenate([n1, n2])
    perm = rng.permutation(n)
    return _finish(_surface_gaussians(rng, pts[perm], nrm[perm]))


def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def make_multi_object_scene(n_objects: int = 8, per_object: int = 150_000, seed_index: int = 2) -> dict:
    """Composition of procedurally placed objects on a ground plane.

    Object 0 is the ground plane; objects 1.. cycle sphere, box, torus, each with a
    seeded scale in [0.7, 1.0], yaw and placement on a jittered grid (spacing 2.6,
    non-overlapping), resting on the plane. Each object has `per_object`
    surface-sampled Gaussians drawn as in the object-scale scene.
    """
    rng = rng_for(seed_index)
    n_obj = max(1, int(n_objects))
    n_place = n_obj - 1
    cols = max(1, int(math.ceil(math.sqrt(max(n_place, 1)))))
    rows = max(1, int(math.ceil(max(n_place, 1) / cols)))
    spacing = 2.6
    half_w = 0.5 * cols * spacing + 1.0
    half_h = 0.5 * rows * spacing + 1.0
    parts = []
    p, nr = _sample_plane(rng, per_object, -half_w, half_w, -half_h, half_h)
    parts.append(_surface_gaussians(rng, p, nr))
    for o in range(n_place):
        r_, c_ = divmod(o, cols)
        cx = (c_ - 0.5 * (cols - 1)) * spacing + rng.uniform(-0.2, 0.2)
        cy = (r_ - 0.5 * (rows - 1)) * spacing + rng.uniform(-0.2, 0.2)
        s = rng.uniform(0.7, 1.0)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        kind = o % 3
        if kind == 0:
            p, nr = _sample_sphere(rng, per_object, (0.0, 0.0, s), s)
        elif kind == 1:
            half = rng.uniform(0.5, 0.9, 3) * s
            p, nr = _sample_box(rng, per_object, half)
            p[:, 2] += half[2]
        else:
            R, r = 0.7 * s, 0.3 * s
            p, nr = _sample_torus(rng, per_object, R, r)
            p[:, 2] += r
        Rz = _rot_z(yaw)
        p = p @ Rz.T + np.array([cx, cy, 0.0])
        nr = nr @ Rz.T
        parts.append(_surface_gaussians(rng, p, nr))
    return _finish(_concat(parts))


def make_scene(name: str, n: int | None = None, n_objects: int | None = None,
               per_object: int | None = None) -> dict:
    """Scene for a preset name, optionally resized (tests use smaller copies)."""
    cfg = PRESETS[name]
    idx = PRESET_INDEX[name]
    if cfg["kind"] == "cube":
        return make_cube_cloud(n or cfg["n"], idx)
    if cfg["kind"] == "object":
        return make_object_scene(n or cfg["n"], idx)
    return make_multi_object_scene(n_objects or cfg["n_objects"], per_object or cfg["per_object"], idx)


def preset_dirs(name: str, K: int | None = None) -> np.ndarray:
    cfg = PRESETS[name]
    return fibonacci_dirs(K or cfg["K"], hemisphere=cfg["dir_mode"] == 1)


def rotated_dirs(K: int, angle: float, hemisphere: bool = True) -> np.ndarray:
    """Fibonacci directions turned by `angle` about the local z axis (the
    normal in hemisphere mode), float32: the per-iteration resampling of the
    incident directions during training."""
    d = fibonacci_dirs(K, hemisphere).astype(np.float64)
    c, s = math.cos(angle), math.sin(angle)
    out = np.stack([c * d[:, 0] - s * d[:, 1], s * d[:, 0] + c * d[:, 1], d[:, 2]], 1)
    return out.astype(np.float32)


def rigid_move(scene: dict, sel, angle_z: float, shift) -> dict:
    """Copy of the scene with Gaussians `sel` (index array or slice) turned by
    angle_z about the vertical axis through their centroid and shifted: the
    edit of an object in a composition (means, rotations and normals move
    together; scales and opacities stay). float32 like the generators."""
    out = {k: v.copy() for k, v in scene.items()}
    mu = scene["mean"][sel].astype(np.float64)
    c = mu.mean(0)
    ca, sa = math.cos(angle_z), math.sin(angle_z)
    R = np.array([[ca, -sa, 0.0], [sa, ca, 0.0], [0.0, 0.0, 1.0]])
    out["mean"][sel] = ((mu - c) @ R.T + c + np.asarray(shift, np.float64)).astype(np.float32)
    out["normal"][sel] = (scene["normal"][sel].astype(np.float64) @ R.T).astype(np.float32)
    # quaternion of the turn, w-first, composed on the left: q' = r q
    rw, rz = math.cos(angle_z / 2), math.sin(angle_z / 2)
    q = scene["quat"][sel].astype(np.float64)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    out["quat"][sel] = np.stack([rw * w - rz * z, rw * x - rz * y, rw * y + rz * x, rw * z + rz * w], 1).astype(np.float32)
    return out


def sample_ray_ids(n: int, K: int, count: int, seed: int) -> np.ndarray:
    """Seeded uniform sample of distinct ray ids r = i*K + k (int64, sorted)."""
    total = n * K
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, total)
    if count * 4 >= total:
        ids = rng.permutation(total)[:count]
    else:
        ids = np.unique(rng.integers(0, total, size=int(count * 1.2) + 16))
        while ids.size < count:
            ids = np.unique(np.concatenate([ids, rng.integers(0, total, size=count)]))
        ids = rng.permutation(ids)[:count]
    return np.sort(ids).astype(np.int64)
