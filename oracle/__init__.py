"""FP64 CPU oracle for point-based ray tracing of 3D Gaussians.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. It shares no code with the HIP
library and never imports it.

`oracle.c` holds the brute-force tracer, the analytic adjoint and the LBVH
reference; `mlp.py` holds the surrogate network reference. This module is the
ctypes binding of `oracle.c` (argument marshalling only).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# default cut parameters: alpha cut 1/255, alpha clamp 0.99, 3-sigma support,
# t_min = 3 * max scale of the source Gaussian
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
SIGMA_CUT = 3.0
TMIN_SCALE = 3.0
KAPPA = 16.0


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("alpha_min", C.c_double), ("alpha_max", C.c_double), ("sigma_cut", C.c_double),
                ("tmin_scale", C.c_double), ("kappa", C.c_double)]


_P = np.ctypeslib.ndpointer
_d = _P(dtype=np.float64, flags="C_CONTIGUOUS")
_f = _P(dtype=np.float32, flags="C_CONTIGUOUS")
_i64 = _P(dtype=np.int64, flags="C_CONTIGUOUS")
_i32 = _P(dtype=np.int32, flags="C_CONTIGUOUS")
_u64 = _P(dtype=np.uint64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        L.or_trace_rays.argtypes = [C.c_int64, _d, _d, _d, _d, _d, C.c_int32, _d, C.c_int32,
                                    C.POINTER(_Params), C.c_int64, _i64, _d, _d, _d, _i32, _i32, _i32, _i32]
        L.or_pair_terms.argtypes = [_d, _d, _d, C.c_int32, _d, C.c_int32, C.POINTER(_Params), C.c_int64, _i64,
                                    C.c_int64, _d, _d, _d, C.c_double, _d, _d, _d, _i32, _i32, _i32]
        L.or_pair_terms.restype = None
        L.or_rays_meeting_boxes.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, C.c_int32, C.c_double,
                                            C.c_int32, _d, _d, _u64]
        L.or_rays_meeting_boxes.restype = None
        L.or_trace_rays.restype = None
        L.or_grad_rays.argtypes = [C.c_int64, _d, _d, _d, _d, _d, C.c_int32, _d, C.c_int32,
                                   C.POINTER(_Params), C.c_int64, _i64, _d, _d, _d, _d, C.c_int32]
        L.or_grad_rays.restype = None
        L.or_rays_meeting_box.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, C.c_int32, C.c_double,
                                          _d, _d, C.c_int64, C.c_int64, _i64]
        L.or_rays_meeting_box.restype = C.c_int64
        L.or_morton63.argtypes = [C.c_int64, _f, _f, _f, _u64]
        L.or_morton63.restype = None
        L.or_radix_tree.argtypes = [C.c_int64, _u64, _i32, _i32, _i32]
        L.or_radix_tree.restype = C.c_int32
        L.or_tree_depth.argtypes = [C.c_int64, _i32, _i32]
        L.or_tree_depth.restype = C.c_int32
        L.or_leaf_boxes.argtypes = [C.c_int64, _d, _d, _d, C.c_double, _d, _d]
        L.or_leaf_boxes.restype = None
        L.or_refit.argtypes = [C.c_int64, _i32, _i32, _d, _d, _d, _d]
        L.or_refit.restype = None
        L.or_peak.argtypes = [_d, _d, _d, _d, _d, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_peak.restype = None
        L.or_whitening.argtypes = [_d, _d, _d]
        L.or_onb.argtypes = [_d, _d, _d]
        L.or_make_ray.argtypes = [_d, _d, _d, C.c_int32, _d, C.c_int32, C.c_double, C.c_int64,
                                  _d, _d, C.POINTER(C.c_double)]
        L.or_max_threads.argtypes = []
        L.or_max_threads.restype = C.c_int32
        L.or_set_threads.argtypes = [C.c_int32]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _scene64(scene: dict):
    n = int(np.asarray(scene["mean"]).shape[0])
    return (n, _f64(scene["mean"]).reshape(-1), _f64(scene["quat"]).reshape(-1),
            _f64(scene["log_scale"]).reshape(-1), _f64(scene["opacity"]).reshape(-1),
            _f64(scene["normal"]).reshape(-1))


def params(alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, sigma_cut=SIGMA_CUT, tmin_scale=TMIN_SCALE,
           kappa=KAPPA) -> _Params:
    return _Params(alpha_min, alpha_max, sigma_cut, tmin_scale, kappa)


def trace_rays(scene: dict, dirs, dir_mode: int, ray_ids, prm: _Params | None = None) -> dict:
    """Brute-force FP64 transmittance of rays r = i*K + k (see oracle.c)."""
    prm = prm or params()
    n, mean, quat, ls, op, nrm = _scene64(scene)
    dirs = _f64(dirs).reshape(-1, 3)
    K = dirs.shape[0]
    ids = np.ascontiguousarray(np.asarray(ray_ids, dtype=np.int64))
    m = ids.shape[0]
    P, lo, hi = np.empty(m), np.empty(m), np.empty(m)
    ninc, namb, ncl, nnc = (np.empty(m, np.int32) for _ in range(4))
    lib().or_trace_rays(n, mean, quat, ls, op, nrm, K, dirs.reshape(-1), int(dir_mode), C.byref(prm),
                        m, ids, P, lo, hi, ninc, namb, ncl, nnc)
    return dict(P=P, V_lo=lo, V_hi=hi, n_incl=ninc, n_amb=namb, n_clamp=ncl, n_near_clamp=nnc)


def pair_terms(scene: dict, dirs, dir_mode: int, ray_ids, j: int, mu=None, quat=None, log_scale=None,
               opacity=None, prm: _Params | None = None) -> dict:
    """Gaussian j's t*, q, alpha, inclusion and ambiguity on each listed ray;
    j's parameters may be overridden (for perturbations)."""
    prm = prm or params()
    n, mean, _, ls, _, nrm = _scene64(scene)
    dirs = _f64(dirs).reshape(-1, 3)
    ids = np.ascontiguousarray(np.asarray(ray_ids, dtype=np.int64))
    m = ids.shape[0]
    mu = _f64(scene["mean"][j] if mu is None else mu)
    qj = _f64(scene["quat"][j] if quat is None else quat)
    lj = _f64(scene["log_scale"][j] if log_scale is None else log_scale)
    oj = float(np.float64(scene["opacity"][j]) if opacity is None else opacity)
    t, q, a = np.empty(m), np.empty(m), np.empty(m)
    inc, amb, nc = np.empty(m, np.int32), np.empty(m, np.int32), np.empty(m, np.int32)
    lib().or_pair_terms(mean, nrm, ls, dirs.shape[0], dirs.reshape(-1), int(dir_mode), C.byref(prm), m, ids,
                        int(j), mu, qj, lj, oj, t, q, a, inc, amb, nc)
    return dict(t=t, q=q, alpha=a, inc=inc, amb=amb, near_clamp=nc)


def rays_meeting_boxes(scene: dict, dirs, dir_mode: int, lo, hi, tmin_scale: float = TMIN_SCALE) -> np.ndarray:
    """uint64 mask per ray r < n*K: bit b set iff ray r's half-line meets box b (<= 64 boxes)."""
    n, mean, _, ls, _, nrm = _scene64(scene)
    dirs = _f64(dirs).reshape(-1, 3)
    lo = _f64(lo).reshape(-1, 3)
    hi = _f64(hi).reshape(-1, 3)
    assert lo.shape == hi.shape and lo.shape[0] <= 64
    mask = np.empty(n * dirs.shape[0], np.uint64)
    lib().or_rays_meeting_boxes(n, mean, nrm, ls, dirs.shape[0], dirs.reshape(-1), int(dir_mode), tmin_scale,
                                lo.shape[0], lo.reshape(-1), hi.reshape(-1), mask)
    return mask


def trace_all(scene: dict, dirs, dir_mode: int, prm: _Params | None = None) -> dict:
    n = int(np.asarray(scene["mean"]).shape[0])
    K = int(np.asarray(dirs).reshape(-1, 3).shape[0])
    return trace_rays(scene, dirs, dir_mode, np.arange(n * K, dtype=np.int64), prm)


def vis_mean(P: np.ndarray, n: int, K: int) -> np.ndarray:
    """Per-Gaussian visibility averaged uniformly over its K directions."""
    return np.asarray(P, dtype=np.float64).reshape(n, K).mean(axis=1)


def grad_rays(scene: dict, dirs, dir_mode: int, ray_ids, weights, prm: _Params | None = None,
              absolute: int = 0) -> dict:
    """Analytic d(sum_s w_s P_s)/d(opacity, mean, log_scale), FP64. absolute=1
    sums the magnitudes of its terms; absolute=2 sums each term's sensitivity
    to binary32 rounding of the ray and of W (an error scale, without kappa)."""
    prm = prm or params()
    n, mean, quat, ls, op, nrm = _scene64(scene)
    dirs = _f64(dirs).reshape(-1, 3)
    ids = np.ascontiguousarray(np.asarray(ray_ids, dtype=np.int64))
    w = _f64(weights).reshape(-1)
    assert w.shape[0] == ids.shape[0]
    go, gm, gl = np.zeros(n), np.zeros(3 * n), np.zeros(3 * n)
    lib().or_grad_rays(n, mean, quat, ls, op, nrm, dirs.shape[0], dirs.reshape(-1), int(dir_mode),
                       C.byref(prm), ids.shape[0], ids, w, go, gm, gl, int(absolute))
    return dict(opacity=go, mean=gm.reshape(n, 3), log_scale=gl.reshape(n, 3))


def rays_meeting_box(scene: dict, dirs, dir_mode: int, lo, hi, always_src: int = -1,
                     tmin_scale: float = TMIN_SCALE) -> np.ndarray:
    n, mean, quat, ls, op, nrm = _scene64(scene)
    dirs = _f64(dirs).reshape(-1, 3)
    cap = 1 << 20
    out = np.empty(cap, np.int64)
    cnt = lib().or_rays_meeting_box(n, mean, nrm, ls, dirs.shape[0], dirs.reshape(-1), int(dir_mode),
                                    tmin_scale, _f64(lo), _f64(hi), int(always_src), cap, out)
    if cnt > cap:
        out = np.empty(cnt, np.int64)
        lib().or_rays_meeting_box(n, mean, nrm, ls, dirs.shape[0], dirs.reshape(-1), int(dir_mode),
                                  tmin_scale, _f64(lo), _f64(hi), int(always_src), cnt, out)
    return out[:cnt].copy()


def morton63(mean_f32) -> tuple:
    """(lo[3], hi[3], keys[N] uint64) in binary32 replay."""
    m = np.ascontiguousarray(np.asarray(mean_f32, dtype=np.float32).reshape(-1))
    n = m.shape[0] // 3
    lo, hi = np.empty(3, np.float32), np.empty(3, np.float32)
    keys = np.empty(n, np.uint64)
    lib().or_morton63(n, m, lo, hi, keys)
    return lo, hi, keys


def sort_keys(keys) -> np.ndarray:
    """Stable ascending order of the keys (ties keep input order)."""
    return np.argsort(np.asarray(keys, dtype=np.uint64), kind="stable").astype(np.int64)


def radix_tree(sorted_keys) -> dict:
    k = np.ascontiguousarray(np.asarray(sorted_keys, dtype=np.uint64))
    n = k.shape[0]
    left = np.zeros(max(n - 1, 1), np.int32)
    right = np.zeros(max(n - 1, 1), np.int32)
    parent = np.zeros(max(2 * n - 1, 1), np.int32)
    lib().or_radix_tree(n, k, left, right, parent)
    return dict(left=left[: max(n - 1, 0)], right=right[: max(n - 1, 0)], parent=parent[: max(2 * n - 1, 0)])


def tree_depth(left, right) -> int:
    left = np.ascontiguousarray(left, dtype=np.int32)
    right = np.ascontiguousarray(right, dtype=np.int32)
    return int(lib().or_tree_depth(left.shape[0] + 1, left if left.size else np.zeros(1, np.int32),
                                   right if right.size else np.zeros(1, np.int32)))


def leaf_boxes(scene: dict, sigma_cut: float = SIGMA_CUT):
    n, mean, quat, ls, _, _ = _scene64(scene)
    lo, hi = np.empty(3 * n), np.empty(3 * n)
    lib().or_leaf_boxes(n, mean, quat, ls, sigma_cut, lo, hi)
    return lo.reshape(n, 3), hi.reshape(n, 3)


def refit(left, right, leaf_lo_sorted, leaf_hi_sorted):
    left = np.ascontiguousarray(left, dtype=np.int32)
    right = np.ascontiguousarray(right, dtype=np.int32)
    n = left.shape[0] + 1
    lo, hi = np.empty(3 * max(n - 1, 1)), np.empty(3 * max(n - 1, 1))
    if n > 1:
        lib().or_refit(n, left, right, _f64(leaf_lo_sorted).reshape(-1), _f64(leaf_hi_sorted).reshape(-1),
                       lo, hi)
    return lo.reshape(-1, 3)[: n - 1], hi.reshape(-1, 3)[: n - 1]


def peak(quat, log_scale, mu, o, d):
    t, q = C.c_double(), C.c_double()
    lib().or_peak(_f64(quat), _f64(log_scale), _f64(mu), _f64(o), _f64(d), C.byref(t), C.byref(q))
    return t.value, q.value


def whitening(quat, log_scale) -> np.ndarray:
    W = np.empty(9)
    lib().or_whitening(_f64(quat), _f64(log_scale), W)
    return W.reshape(3, 3)


def onb(nrm):
    b1, b2 = np.empty(3), np.empty(3)
    lib().or_onb(_f64(nrm), b1, b2)
    return b1, b2


def make_ray(scene: dict, dirs, dir_mode: int, r: int, tmin_scale: float = TMIN_SCALE):
    n, mean, quat, ls, op, nrm = _scene64(scene)
    dirs = _f64(dirs).reshape(-1, 3)
    o, d, tm = np.empty(3), np.empty(3), C.c_double()
    lib().or_make_ray(mean, nrm, ls, dirs.shape[0], dirs.reshape(-1), int(dir_mode), tmin_scale, int(r),
                      o, d, C.byref(tm))
    return o, d, tm.value


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().or_max_threads())


def set_threads(t: int) -> None:
    lib().or_set_threads(int(t))
