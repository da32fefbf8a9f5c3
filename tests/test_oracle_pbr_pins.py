"""Pins of the FP64 shading oracle (Sec. 3.3, Eq. (7)-(10)) against facts that
do not come from its own formulas: normalisation of the GGX distribution, the
weak white furnace identity, limits of Schlick and Smith, orthonormality of the
SH basis, texel-centre and seam behaviour of the environment lookup, the
direction frame of the visibility rays, and closed forms of the sum for
uniform light."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import pbr
from workloads import materials, scenes


def _gl_sphere(n_mu=64, n_phi=128, hemisphere=False, lo=None):
    """Product rule on the sphere (cos(theta) >= lo; lo = 0 for the hemisphere):
    Gauss-Legendre in cos(theta), uniform in phi."""
    x, wx = np.polynomial.legendre.leggauss(n_mu)
    if lo is None:
        lo = 0.0 if hemisphere else -1.0
    mu = lo + (x + 1.0) * (1.0 - lo) / 2.0
    wmu = wx * (1.0 - lo) / 2.0
    phi = (np.arange(n_phi) + 0.5) * 2.0 * math.pi / n_phi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    s = np.sqrt(1.0 - M * M)
    w = np.stack([s * np.cos(P), s * np.sin(P), M], -1).reshape(-1, 3)
    wt = (wmu[:, None] * np.full(n_phi, 2.0 * math.pi / n_phi)[None]).reshape(-1)
    return w, wt


@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.5, 1.0])
def test_ggx_distribution_is_normalised(alpha):
    # the projected microfacet area integrates to one: int D(h) (n.h) dw_h = 1
    val, _ = integrate.quad(lambda mu: float(pbr.ggx_D(mu, alpha)) * mu * 2.0 * math.pi, 0.0, 1.0,
                            points=[1.0 - alpha], limit=400, epsabs=1e-12)
    assert abs(val - 1.0) < 1e-8


@pytest.mark.parametrize("alpha,theta_o", [(0.3, 0.0), (0.3, 1.0), (0.7, 0.5), (1.0, 1.3)])
def test_weak_white_furnace(alpha, theta_o):
    # int D(h) G1(w_o) / (4 |n.w_o|) dw_i = 1 (Heitz 2014): the 1/4 Jacobian of
    # the half vector, D and G1 together
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([math.sin(theta_o), 0.0, math.cos(theta_o)])
    # microfacet normals exist only above the surface: n.(w_i + w_o) > 0, i.e.
    # cos(theta_i) > -cos(theta_o); integrate over exactly that cap
    w, wt = _gl_sphere(400, 400, lo=-wo[2])
    h = pbr._unit(w + wo)
    integrand = pbr.ggx_D(np.maximum(h @ n, 0.0), alpha) * pbr.smith_G1(wo @ n, alpha) / (4.0 * (wo @ n))
    assert abs(np.sum(integrand * wt) - 1.0) < 1e-4


def test_specular_lobe_of_a_smooth_mirror_reflects_almost_everything():
    # r = 0.2 (alpha 0.04), F = 1, normal incidence: the directional albedo of
    # the full lobe is just below one (a missing or extra factor of 4 fails)
    n = np.array([0.0, 0.0, 1.0])
    w, wt = _gl_sphere(1200, 64, hemisphere=True)
    val = np.sum(pbr.specular_cos(n, n, w, 0.2, 1.0) * wt)
    assert 0.98 < val <= 1.0 + 1e-6


def test_schlick_and_smith_limits():
    assert pbr.schlick_F(1.0, 0.04) == pytest.approx(0.04, abs=1e-15)
    assert pbr.schlick_F(0.0, 0.04) == pytest.approx(1.0, abs=1e-15)
    for a in (0.01, 0.3, 1.0):
        assert pbr.smith_G1(1.0, a) == pytest.approx(1.0, abs=1e-14)
        assert pbr.smith_G1(1e-9, a) < 1e-6
    assert pbr.smith_G1(0.2, 0.0) == pytest.approx(1.0, abs=1e-14)   # perfectly smooth: no masking


def test_sh_basis_is_orthonormal():
    w, wt = _gl_sphere(16, 32)
    Y = pbr.sh_basis(w)
    G = (Y * wt[:, None]).T @ Y
    assert np.allclose(G, np.eye(9), atol=1e-12)


def test_env_lookup_texel_centres_seam_and_poles():
    env = materials.make_env(1).astype(np.float64)
    r, c = np.meshgrid(np.arange(16), np.arange(32), indexing="ij")
    theta = (r + 0.5) * math.pi / 16
    phi = (c + 0.5) * 2 * math.pi / 32 - math.pi
    w = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)
    assert np.allclose(pbr.env_lookup(env, w), env, atol=1e-12)
    # constant map -> constant everywhere
    w2 = scenes.fibonacci_dirs(500, False)
    assert np.allclose(pbr.env_lookup(np.full((16, 32, 3), 2.5), w2), 2.5, atol=1e-14)
    # continuous across the azimuth seam at -pi / pi
    eps = 1e-9
    a = pbr.env_lookup(env, np.array([math.cos(math.pi - eps), math.sin(math.pi - eps), 0.3]))
    b = pbr.env_lookup(env, np.array([math.cos(-math.pi + eps), math.sin(-math.pi + eps), 0.3]))
    assert np.allclose(a, b, atol=1e-6)
    # halfway between two texel centres of one row: their average
    wm = np.array([math.sin(theta[3, 0]) * math.cos(-math.pi + 2 * math.pi / 32),
                   math.sin(theta[3, 0]) * math.sin(-math.pi + 2 * math.pi / 32), math.cos(theta[3, 0])])
    assert np.allclose(pbr.env_lookup(env, wm), 0.5 * (env[3, 0] + env[3, 1]), atol=1e-12)
    # +z pole: row 0 only (clamped), halfway between columns 15 and 16 (azimuth 0)
    assert np.allclose(pbr.env_lookup(env, np.array([0.0, 0.0, 1.0])), 0.5 * (env[0, 15] + env[0, 16]), atol=1e-12)


def test_directions_match_the_visibility_rays():
    sc = scenes.make_object_scene(200, 1)
    dirs = scenes.fibonacci_dirs(16, True)
    w = pbr.directions(sc["normal"], dirs, 1)
    for r in (0, 5, 17, 200 * 16 - 1, 1234):
        _, d, _ = oracle.make_ray(sc, dirs, 1, r)
        assert np.allclose(w[r // 16, r % 16], d, atol=1e-14)


def _uniform_setup(n=50, K=64, E=1.7, seed=0):
    sc = scenes.make_object_scene(n, 1)
    m = materials.make_materials(n, seed)
    env = np.full((16, 32, 3), E)
    return sc, m, env, scenes.fibonacci_dirs(K, True)


def test_diffuse_part_under_uniform_light_is_albedo_times_light():
    # Fibonacci hemisphere: sum_k z_k = K / 2, so sum_k cos * 2 pi / K = pi
    # (to the float32 rounding of the direction table, ~1e-9), and the diffuse
    # part of Eq. (10) is b * E
    sc, m, env, dirs = _uniform_setup()
    V = np.ones((50, 64))
    sh0 = np.zeros((50, 9, 3))
    c1, _ = pbr.shade(sc["mean"], sc["normal"], dirs, 1, V, m["albedo"], m["roughness"], sh0, env,
                      materials.CAMERA)
    c0, _ = pbr.shade(sc["mean"], sc["normal"], dirs, 1, V, np.zeros((50, 3)), m["roughness"], sh0, env,
                      materials.CAMERA)
    assert np.allclose(c1 - c0, m["albedo"].astype(np.float64) * 1.7, rtol=1e-8, atol=1e-12)


def test_constant_indirect_light_and_zero_visibility():
    # V = 0 and only the DC SH coefficient s: L = s Y_00 = s / (2 sqrt(pi)) in
    # every direction, so the diffuse part is b s / (2 sqrt(pi))
    sc, m, env, dirs = _uniform_setup()
    sh = np.zeros((50, 9, 3))
    sh[:, 0, :] = 0.8
    V = np.zeros((50, 64))
    c1, _ = pbr.shade(sc["mean"], sc["normal"], dirs, 1, V, m["albedo"], m["roughness"], sh, env, materials.CAMERA)
    c0, _ = pbr.shade(sc["mean"], sc["normal"], dirs, 1, V, np.zeros((50, 3)), m["roughness"], sh, env,
                      materials.CAMERA)
    assert np.allclose(c1 - c0, m["albedo"].astype(np.float64) * 0.8 / (2.0 * math.sqrt(math.pi)), rtol=1e-8,
                       atol=1e-12)
    # and the environment does not enter when nothing is visible
    c2, _ = pbr.shade(sc["mean"], sc["normal"], dirs, 1, V, m["albedo"], m["roughness"], sh, env * 3.0,
                      materials.CAMERA)
    assert np.array_equal(c1, c2)


def test_sum_is_linear_in_visibility_and_brute_force_on_a_tiny_case():
    sc = scenes.make_object_scene(3, 1)
    m = materials.make_materials(3, 2)
    env = materials.make_env(2).astype(np.float64)
    dirs = scenes.fibonacci_dirs(5, True)
    V = materials.make_visibility(3, 5, 3).astype(np.float64)
    c, _ = pbr.shade(sc["mean"], sc["normal"], dirs, 1, V, m["albedo"], m["roughness"], m["sh"], env,
                     materials.CAMERA)
    # term by term with the ray directions of the C oracle and a hand-built
    # half vector, one direction at a time
    sc64 = {k: v.astype(np.float64) for k, v in sc.items()}
    m64 = {k: v.astype(np.float64) for k, v in m.items()}
    cam = materials.CAMERA.astype(np.float64)
    for i in range(3):
        n = sc64["normal"][i] / np.linalg.norm(sc64["normal"][i])
        wo = cam - sc64["mean"][i]
        wo = wo / np.linalg.norm(wo)
        acc = np.zeros(3)
        for k in range(5):
            _, w, _ = oracle.make_ray(sc, dirs, 1, i * 5 + k)
            ci = float(w @ n)
            light = V[i, k] * pbr.env_lookup(env, w) + pbr.sh_basis(w) @ m64["sh"][i]
            h = (w + wo) / np.linalg.norm(w + wo)
            a = float(m64["roughness"][i]) ** 2
            spec = 0.0
            if ci > 0 and wo @ n > 0:
                spec = float(pbr.ggx_D(h @ n, a) * pbr.schlick_F(wo @ h, 0.04) * pbr.smith_G1(ci, a) *
                             pbr.smith_G1(wo @ n, a) / (4.0 * ci * (wo @ n)))
            acc += (m64["albedo"][i] / math.pi + spec) * light * max(ci, 0.0) * 2 * math.pi / 5
        assert np.allclose(c[i], acc, rtol=1e-12, atol=1e-14)


# ---- visibility compressed to SH (oracle/vis_sh.py) ----

from oracle import vis_sh  # noqa: E402


def test_sh_projection_of_constant_and_of_a_cap():
    K = 256
    dirs = scenes.fibonacci_dirs(K, True)
    # constant visibility c: v_00 = c Y_00 2 pi = c sqrt(pi) (the weights sum to 2 pi exactly)
    v = vis_sh.project(np.full((1, K), 0.7), dirs, 1)
    assert v[0, 0] == pytest.approx(0.7 * math.sqrt(math.pi), rel=1e-12)
    # visibility 1 on the cap z > 1/2 (exactly the first K/2 Fibonacci samples):
    # v_00 = Y_00 pi and v_10 = sqrt(3/(4 pi)) sum z dw = sqrt(3/(4 pi)) 3 pi / 4
    # (the equal-area z spacing integrates z exactly)
    cap = (dirs[:, 2].astype(np.float64) > 0.5).astype(np.float64)[None]
    assert cap.sum() == K // 2
    v = vis_sh.project(cap, dirs, 1)
    assert v[0, 0] == pytest.approx(0.5 / math.sqrt(math.pi) * math.pi, rel=1e-6)
    assert v[0, 2] == pytest.approx(math.sqrt(3 / (4 * math.pi)) * 0.75 * math.pi, rel=1e-6)


def test_sh_projection_recovers_each_basis_function():
    # sphere mode with many directions: projecting Y_j returns the unit vector e_j
    dirs = scenes.fibonacci_dirs(40_000, False)
    Y = pbr.sh_basis(dirs.astype(np.float64) / np.linalg.norm(dirs.astype(np.float64), axis=1, keepdims=True))
    v = vis_sh.project(Y.T, dirs, 0)
    assert np.allclose(v, np.eye(9), atol=2e-4)


def test_sh_projection_bounds_bracket_every_visibility_in_between():
    rng = np.random.default_rng(3)
    dirs = scenes.fibonacci_dirs(64, True)
    lo = rng.uniform(0, 0.5, (20, 64))
    hi = lo + rng.uniform(0, 0.3, (20, 64))
    blo, bhi = vis_sh.project_bounds(lo, hi, dirs, 1)
    for _ in range(20):
        v = vis_sh.project(lo + rng.uniform(0, 1, lo.shape) * (hi - lo), dirs, 1)
        assert np.all(v >= blo - 1e-12) and np.all(v <= bhi + 1e-12)
