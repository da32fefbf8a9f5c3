"""Pins of the FP64 oracle against closed forms, library routines and invariants.

Each test ties one part of the oracle to something other than its own formulas:
a dense numerical search, scipy's rotation convention, a hand-derived value, or
a structural property fixed by the paper (order independence, Sec. 4.1).
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.transform import Rotation

import oracle
from workloads import scenes


def _sigma_inv(quat_wxyz, log_scale):
    """Sigma^-1 through scipy's rotation (x,y,z,w order) and a matrix inverse."""
    w, x, y, z = quat_wxyz
    R = Rotation.from_quat([x, y, z, w]).as_matrix()
    S = np.diag(np.exp(log_scale))
    Sigma = R @ S @ S.T @ R.T
    return np.linalg.inv(Sigma), Sigma


def _one_gaussian_scene(mu, quat, ls, opac):
    return dict(mean=np.asarray(mu, np.float64)[None], quat=np.asarray(quat, np.float64)[None],
                log_scale=np.asarray(ls, np.float64)[None], opacity=np.asarray([opac], np.float64),
                normal=np.asarray([[0.0, 0.0, 1.0]]))


def _scene_from(list_of_g):
    keys = ["mean", "quat", "log_scale", "opacity", "normal"]
    return {k: np.asarray([g[k] for g in list_of_g], np.float64) for k in keys}


def _g(mu, quat=(1, 0, 0, 0), ls=(math.log(0.05),) * 3, o=0.5, n=(0, 0, 1)):
    return dict(mean=mu, quat=quat, log_scale=ls, opacity=o, normal=n)


# ---------------------------------------------------------------------------
# peak point, Eq. (13)-(14)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_peak_matches_dense_search(seed):
    rng = np.random.default_rng(100 + seed)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    ls = rng.uniform(math.log(0.01), math.log(0.3), 3)
    mu = rng.uniform(-1, 1, 3)
    o = rng.uniform(-1, 1, 3)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    Si, _ = _sigma_inv(q, ls)

    def expo(t):
        x = o + t * d - mu
        return float(x @ Si @ x)

    ts = np.linspace(-10, 10, 200001)
    X = o[None] + ts[:, None] * d[None] - mu[None]
    vals = np.einsum("ni,ij,nj->n", X, Si, X)
    t0 = ts[np.argmin(vals)]
    res = minimize_scalar(expo, bracket=(t0 - 1e-3, t0, t0 + 1e-3), tol=1e-14)
    t_star, q_val = oracle.peak(q, ls, mu, o, d)
    assert abs(t_star - res.x) <= 1e-6 * max(1.0, abs(res.x))
    assert abs(q_val - res.fun) <= 1e-9 * max(1.0, res.fun)


def test_peak_isotropic_is_orthogonal_projection():
    rng = np.random.default_rng(7)
    s = 0.07
    for _ in range(20):
        mu, o = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        q = rng.normal(size=4)
        t_star, qv = oracle.peak(q / np.linalg.norm(q), [math.log(s)] * 3, mu, o, d)
        t_ref = float(d @ (mu - o))
        foot = o + t_ref * d
        assert abs(t_star - t_ref) < 1e-12
        assert abs(qv - float(np.sum((mu - foot) ** 2)) / s**2) < 1e-9 * max(1, qv)


def test_printed_sigma_form_differs_from_peak_for_anisotropic_gaussian():
    """Eq. (14) as printed weights by Sigma; the peak of Eq. (1) needs Sigma^-1.
    For an anisotropic Gaussian the two differ and the dense search sides with
    Sigma^-1 (the reading the oracle takes)."""
    q = np.array([0.9, 0.3, -0.2, 0.25])
    q /= np.linalg.norm(q)
    ls = np.log([0.02, 0.2, 0.05])
    mu, o = np.array([0.3, -0.1, 0.8]), np.array([-0.5, 0.2, -0.4])
    d = np.array([0.6, -0.2, 0.75])
    d /= np.linalg.norm(d)
    Si, Sigma = _sigma_inv(q, ls)
    t_printed = float((mu - o) @ Sigma @ d / (d @ Sigma @ d))
    t_inv = float((mu - o) @ Si @ d / (d @ Si @ d))
    t_star, _ = oracle.peak(q, ls, mu, o, d)
    ts = np.linspace(-5, 5, 400001)
    X = o[None] + ts[:, None] * d[None] - mu[None]
    t_dense = ts[np.argmin(np.einsum("ni,ij,nj->n", X, Si, X))]
    assert abs(t_printed - t_inv) > 1e-2
    assert abs(t_star - t_inv) < 1e-10
    assert abs(t_dense - t_inv) < 1e-4


def test_whitening_matches_scipy_rotation():
    rng = np.random.default_rng(3)
    for _ in range(10):
        q = rng.normal(size=4)
        ls = rng.uniform(-4, 0, 3)
        W = oracle.whitening(q, ls)
        Si, _ = _sigma_inv(q / np.linalg.norm(q), ls)
        assert np.allclose(W.T @ W, Si, rtol=1e-12, atol=1e-9 * np.abs(Si).max())


# ---------------------------------------------------------------------------
# transmittance (Sec. 4.1, Eq. (15)) and the cuts
# ---------------------------------------------------------------------------

def _trace_single_ray(scene, src, direction, prm=None):
    """Trace the one ray leaving Gaussian `src` along `direction` (sphere mode)."""
    dirs = np.asarray([direction], np.float64)
    return oracle.trace_rays(scene, dirs, 0, [src * 1], prm or oracle.params())


def test_no_occluder_gives_unit_transmittance():
    sc = _scene_from([_g([0, 0, 0])])
    r = _trace_single_ray(sc, 0, [0, 0, 1])
    assert r["P"][0] == 1.0 and r["n_incl"][0] == 0
    # occluders behind the ray or far to the side do not count
    sc = _scene_from([_g([0, 0, 0]), _g([0, 0, -1.0]), _g([1.0, 0, 1.0])])
    r = _trace_single_ray(sc, 0, [0, 0, 1])
    assert r["P"][0] == 1.0


def test_ray_through_mean_has_alpha_equal_opacity():
    sc = _scene_from([_g([0, 0, 0]), _g([0, 0, 1.0], o=0.37)])
    r = _trace_single_ray(sc, 0, [0, 0, 1])
    assert abs(r["P"][0] - (1 - 0.37)) < 1e-15


@pytest.mark.parametrize("off_sigma", [0.0, 0.5, 1.5, 2.5, 2.99, 3.01, 4.0])
def test_single_occluder_closed_form(off_sigma):
    s = 0.05
    ls = (math.log(s),) * 3
    o_val = 0.8
    sc = _scene_from([_g([0, 0, 0]), _g([off_sigma * s, 0, 1.0], ls=ls, o=o_val)])
    r = _trace_single_ray(sc, 0, [0, 0, 1])
    qv = off_sigma**2
    alpha = o_val * math.exp(-qv / 2)
    expect = 1 - min(alpha, 0.99) if (qv <= 9 and alpha >= 1 / 255) else 1.0
    assert abs(r["P"][0] - expect) < 1e-14


def test_alpha_cut_and_clamp():
    # opacity so low that alpha < 1/255 even at the peak: excluded
    sc = _scene_from([_g([0, 0, 0]), _g([0, 0, 1], o=0.9 / 255)])
    assert _trace_single_ray(sc, 0, [0, 0, 1])["P"][0] == 1.0
    # opacity above the clamp: alpha = 0.99
    sc = _scene_from([_g([0, 0, 0]), _g([0, 0, 1], o=0.999)])
    assert abs(_trace_single_ray(sc, 0, [0, 0, 1])["P"][0] - 0.01) < 1e-15


def test_tmin_cut_uses_source_max_scale():
    # source max scale 0.1 -> t_min = 0.3; occluder peak at t = 0.25 is skipped
    src = _g([0, 0, 0], ls=(math.log(0.1), math.log(0.01), math.log(0.02)))
    sc = _scene_from([src, _g([0, 0, 0.25], o=0.6)])
    assert _trace_single_ray(sc, 0, [0, 0, 1])["P"][0] == 1.0
    sc = _scene_from([src, _g([0, 0, 0.35], o=0.6)])
    assert abs(_trace_single_ray(sc, 0, [0, 0, 1])["P"][0] - 0.4) < 1e-15


def test_source_gaussian_excluded_by_index():
    # a second Gaussian sitting exactly at the source mean with a huge scale
    # would be hit; the source itself never is
    src = _g([0, 0, 0], ls=(math.log(0.01),) * 3, o=0.9)
    sc = _scene_from([src])
    assert _trace_single_ray(sc, 0, [0, 0, 1])["P"][0] == 1.0


def test_duplicate_occluder_squares():
    a = _g([0.01, 0, 1.0], o=0.45)
    sc1 = _scene_from([_g([0, 0, 0]), a])
    sc2 = _scene_from([_g([0, 0, 0]), a, a])
    p1 = _trace_single_ray(sc1, 0, [0, 0, 1])["P"][0]
    p2 = _trace_single_ray(sc2, 0, [0, 0, 1])["P"][0]
    assert abs(p2 - p1 * p1) < 1e-15


def test_order_independence_under_permutation():
    """Sec. 4.1: the order in which Gaussians are met does not change T."""
    sc = scenes.make_cube_cloud(300, 0)
    dirs = scenes.fibonacci_dirs(16, hemisphere=False)
    n, K = 300, 16
    base = oracle.trace_all(sc, dirs, 0)["P"].reshape(n, K)
    perm = np.random.default_rng(5).permutation(n)
    sc2 = {k: v[perm] for k, v in sc.items()}
    got = oracle.trace_all(sc2, dirs, 0)["P"].reshape(n, K)
    assert np.allclose(got, base[perm], rtol=0, atol=1e-14)


def test_ambiguity_bounds_bracket_the_definition():
    sc = scenes.make_cube_cloud(400, 0)
    dirs = scenes.fibonacci_dirs(32, hemisphere=False)
    r = oracle.trace_all(sc, dirs, 0)
    assert np.all(r["V_lo"] <= r["P"] + 1e-15) and np.all(r["P"] <= r["V_hi"] + 1e-15)
    clean = r["n_amb"] == 0
    assert np.array_equal(r["V_lo"][clean], r["P"][clean])
    assert np.array_equal(r["V_hi"][clean], r["P"][clean])


# ---------------------------------------------------------------------------
# directions and frames (Sec. 3.3, Sec. 4.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K,hemi", [(64, False), (256, True), (7, True), (1, False)])
def test_fibonacci_dirs_unit_and_equal_area(K, hemi):
    d = scenes.fibonacci_dirs(K, hemi).astype(np.float64)
    assert d.shape == (K, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    z = d[:, 2]
    # equal-area bands: consecutive heights are uniformly spaced
    if K > 1:
        step = np.diff(z)
        assert np.allclose(step, step[0], atol=1e-6)
        assert abs(abs(step[0]) - ((1.0 if hemi else 2.0) / K)) < 1e-6
    if hemi:
        assert np.all(z > 0)
    # golden-angle azimuth increments
    if K > 2:
        phi = np.arctan2(d[:, 1], d[:, 0])
        dphi = np.mod(np.diff(phi), 2 * math.pi)
        assert np.allclose(dphi, math.pi * (3 - math.sqrt(5)), atol=1e-5)


def test_onb_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(11)
    ns = rng.normal(size=(200, 3))
    ns = np.concatenate([ns, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 0, -1 + 1e-12]]])
    for n in ns:
        n = n / np.linalg.norm(n)
        b1, b2 = oracle.onb(n)
        M = np.stack([b1, b2, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(b1, b2), n, atol=1e-12)


def test_hemisphere_rays_leave_the_surface():
    sc = scenes.make_object_scene(50, 1)
    dirs = scenes.fibonacci_dirs(32, True)
    for r in range(0, 50 * 32, 7):
        o, d, tmin = oracle.make_ray(sc, dirs, 1, r)
        i = r // 32
        nrm = sc["normal"][i].astype(np.float64)
        assert np.allclose(o, sc["mean"][i].astype(np.float64))
        assert abs(np.linalg.norm(d) - 1) < 1e-14
        assert d @ nrm / np.linalg.norm(nrm) > 0
        assert abs(tmin - 3 * math.exp(sc["log_scale"][i].astype(np.float64).max())) < 1e-15


# ---------------------------------------------------------------------------
# LBVH reference (Sec. 4.1: binary radix tree after Karras 2012)
# ---------------------------------------------------------------------------

def test_morton_hand_placed_points():
    pts = np.array([[0, 0, 0], [1, 1, 1], [0.5, 0.25, 0.75]], np.float32)
    lo, hi, keys = oracle.morton63(pts)
    assert np.array_equal(lo, [0, 0, 0]) and np.array_equal(hi, [1, 1, 1])
    assert int(keys[0]) == 0
    assert int(keys[1]) == (1 << 63) - 1
    # x = 2^20 -> bit 62; y = 2^19 -> bit 58; z = 2^20 + 2^19 -> bits 60, 57
    assert int(keys[2]) == (1 << 62) | (1 << 58) | (1 << 60) | (1 << 57)


def test_morton_degenerate_axis_and_single_point():
    pts = np.array([[0.25, 3.0, -1.0], [0.75, 3.0, -1.0]], np.float32)
    lo, hi, keys = oracle.morton63(pts)
    # y and z have zero extent -> code 0; x spans [0.25, 0.75]
    assert int(keys[0]) == 0
    assert int(keys[1]) == int(sum(1 << (3 * b + 2) for b in range(21)))
    _, _, k1 = oracle.morton63(np.array([[5, 5, 5]], np.float32))
    assert int(k1[0]) == 0


def test_morton_matches_float32_numpy_replay():
    sc = scenes.make_object_scene(5000, 1)
    m = sc["mean"]
    lo, hi, keys = oracle.morton63(m)
    den = (hi - lo).astype(np.float32)
    u = ((m - lo).astype(np.float32) / den).astype(np.float32)
    c = np.clip(np.floor((u * np.float32(2097152.0)).astype(np.float32)), 0, 2097151).astype(np.uint64)
    ref = np.zeros(len(m), np.uint64)
    for b in range(21):
        for a in range(3):
            ref |= ((c[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + 2 - a)
    assert np.array_equal(keys, ref)


def test_radix_tree_small_cases():
    t1 = oracle.radix_tree(np.array([7], np.uint64))
    assert t1["left"].size == 0 and list(t1["parent"]) == [-1]
    t2 = oracle.radix_tree(np.array([3, 9], np.uint64))
    assert list(t2["left"]) == [~0] and list(t2["right"]) == [~1]
    assert list(t2["parent"]) == [-1, 0, 0]
    # five equal keys: the tree is the radix tree on the position bits
    t5 = oracle.radix_tree(np.full(5, 42, np.uint64))
    assert list(t5["left"]) == [3, ~0, ~2, 1]
    assert list(t5["right"]) == [~4, ~1, ~3, 2]
    assert list(t5["parent"]) == [-1, 3, 3, 0, 1, 1, 2, 2, 0]


def _check_radix_tree(keys, tree):
    """Binary radix tree with Karras numbering, checked from its definition."""
    n = len(keys)
    left, right, parent = tree["left"], tree["right"], tree["parent"]
    aug = [(int(k) << 32) | i for i, k in enumerate(keys)]
    seen_leaf = np.zeros(n, int)
    seen_node = np.zeros(n - 1, int)

    def ranges(node):
        if node < 0:
            m = ~node
            seen_leaf[m] += 1
            return m, m
        seen_node[node] += 1
        f1, l1 = ranges(int(left[node]))
        f2, l2 = ranges(int(right[node]))
        assert l1 + 1 == f2, "children ranges must be adjacent"
        f, l = f1, l2
        assert node in (f, l), "Karras numbering: an internal node sits at one end of its range"
        b = (aug[f] ^ aug[l]).bit_length() - 1
        # every key in the range shares the bits above b; left half has 0 at b
        for m in range(f, l + 1):
            assert (aug[m] >> (b + 1)) == (aug[f] >> (b + 1))
            assert ((aug[m] >> b) & 1) == (0 if m <= l1 else 1)
        for ch, side in ((int(left[node]), 0), (int(right[node]), 1)):
            idx = (n - 1 + ~ch) if ch < 0 else ch
            assert parent[idx] == node
        return f, l

    import sys
    sys.setrecursionlimit(10000)
    f, l = ranges(0)
    assert (f, l) == (0, n - 1) and parent[0] == -1
    assert np.all(seen_leaf == 1) and np.all(seen_node == 1)


@pytest.mark.parametrize("seed", range(5))
def test_radix_tree_random_keys_with_duplicates(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 300))
    keys = np.sort(rng.integers(0, 1 << int(rng.integers(2, 63)), size=n).astype(np.uint64))
    _check_radix_tree(keys, oracle.radix_tree(keys))


def test_radix_tree_on_scene_keys_and_depth_bound():
    sc = scenes.make_object_scene(3000, 1)
    _, _, keys = oracle.morton63(sc["mean"])
    order = oracle.sort_keys(keys)
    sk = keys[order]
    tree = oracle.radix_tree(sk)
    _check_radix_tree(sk, tree)
    # every level consumes at least one bit of the 95-bit augmented key
    assert oracle.tree_depth(tree["left"], tree["right"]) <= 95


def test_leaf_boxes_contain_the_3sigma_ellipsoid():
    sc = scenes.make_cube_cloud(50, 0)
    lo, hi = oracle.leaf_boxes(sc)
    rng = np.random.default_rng(1)
    u = rng.normal(size=(20000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for i in range(50):
        q = sc["quat"][i].astype(np.float64)
        w, x, y, z = q / np.linalg.norm(q)
        R = Rotation.from_quat([x, y, z, w]).as_matrix()
        s = np.exp(sc["log_scale"][i].astype(np.float64))
        pts = sc["mean"][i].astype(np.float64) + 3.0 * (u * s) @ R.T
        assert np.all(pts >= lo[i] - 1e-12) and np.all(pts <= hi[i] + 1e-12)
        # tight: the sampled extremes come within 1% of the box faces
        ext = hi[i] - lo[i]
        assert np.all(pts.min(0) - lo[i] < 0.01 * ext)
        assert np.all(hi[i] - pts.max(0) < 0.01 * ext)


def test_refit_is_union_of_children():
    sc = scenes.make_cube_cloud(200, 0)
    _, _, keys = oracle.morton63(sc["mean"])
    order = oracle.sort_keys(keys)
    tree = oracle.radix_tree(keys[order])
    llo, lhi = oracle.leaf_boxes(sc)
    nlo, nhi = oracle.refit(tree["left"], tree["right"], llo[order], lhi[order])
    # the root box is the box of all leaves
    assert np.array_equal(nlo[0], llo.min(0)) and np.array_equal(nhi[0], lhi.max(0))


# ---------------------------------------------------------------------------
# analytic adjoint vs finite differences of the oracle forward
# ---------------------------------------------------------------------------

def _fd_scene():
    """A few occluders stacked along the +z rays of Gaussian 0, well away from the cuts."""
    rng = np.random.default_rng(21)
    gs = [_g([0, 0, 0], ls=(math.log(0.02),) * 3, o=0.5)]
    for z in (0.4, 0.7, 1.0, 1.3):
        q = rng.normal(size=4)
        gs.append(_g([rng.uniform(-0.03, 0.03), rng.uniform(-0.03, 0.03), z], quat=q / np.linalg.norm(q),
                     ls=np.log(rng.uniform(0.04, 0.09, 3)), o=rng.uniform(0.2, 0.8)))
    return _scene_from(gs)


def test_adjoint_matches_central_differences():
    sc = _fd_scene()
    n = sc["mean"].shape[0]
    dirs = np.array([[0, 0, 1.0], [0.03, 0.02, 1.0], [-0.02, 0.04, 1.0]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rays = np.arange(n * 3, dtype=np.int64)
    w = np.random.default_rng(2).uniform(-1, 1, rays.size)
    g = oracle.grad_rays(sc, dirs, 0, rays, w)

    def F(s):
        return float(np.dot(w, oracle.trace_rays(s, dirs, 0, rays)["P"]))

    h = 1e-6
    checked = 0
    for name, shape in (("opacity", (n,)), ("mean", (n, 3)), ("log_scale", (n, 3))):
        for idx in np.ndindex(*shape):
            sp = {k: v.copy() for k, v in sc.items()}
            sm = {k: v.copy() for k, v in sc.items()}
            sp[name][idx] += h
            sm[name][idx] -= h
            fd = (F(sp) - F(sm)) / (2 * h)
            an = g[name][idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (name, idx, fd, an)
            checked += abs(fd) > 1e-3
    assert checked >= 10


def test_single_occluder_opacity_derivative_closed_form():
    s = 0.05
    off = 1.2
    sc = _scene_from([_g([0, 0, 0]), _g([off * s, 0, 1.0], ls=(math.log(s),) * 3, o=0.6)])
    g = oracle.grad_rays(sc, np.array([[0, 0, 1.0]]), 0, np.array([0], np.int64), np.array([1.0]))
    # T = 1 - o exp(-q/2) -> dT/do = -exp(-q/2), dT/dls = -o exp(-q/2) * q (isotropic scale)
    e = math.exp(-off**2 / 2)
    assert abs(g["opacity"][1] + e) < 1e-14
    assert abs(g["log_scale"][1].sum() + 0.6 * e * off**2) < 1e-13
    # q = (mu_x / s)^2 along the +z ray through x = 0, so dq/dmu_x = 2 off / s and
    # dT/dmu_x = o e^{-q/2} off / s: moving the occluder away raises T
    assert abs(g["mean"][1][0] - (0.6 * e * off / s)) < 1e-12
    # the source mean moves the ray origin: equal and opposite in x
    assert abs(g["mean"][0][0] + g["mean"][1][0]) < 1e-12
