"""Seeded synthetic shading inputs: per-Gaussian albedo, roughness and
indirect-light SH coefficients, a 16 x 32 environment map and a camera
position. Random numbers only; no shading arithmetic lives here."""
from __future__ import annotations

import numpy as np

ENV_ROWS, ENV_COLS = 16, 32


def make_materials(n: int, seed: int = 0) -> dict:
    """albedo U[0,1]^3, roughness U[0.05, 1], SH: DC U[0, 0.5] per channel and
    higher orders N(0, 0.1^2) (float32)."""
    rng = np.random.Generator(np.random.PCG64(31337 + seed))
    albedo = rng.uniform(0.0, 1.0, (n, 3))
    roughness = rng.uniform(0.05, 1.0, n)
    sh = rng.normal(0.0, 0.1, (n, 9, 3))
    sh[:, 0, :] = rng.uniform(0.0, 0.5, (n, 3))
    return dict(albedo=albedo.astype(np.float32), roughness=roughness.astype(np.float32),
                sh=sh.astype(np.float32))


def make_env(seed: int = 0) -> np.ndarray:
    """[16, 32, 3] sky-like map: bright bluish upper half, dim lower half,
    texel noise and one bright sun texel (float32)."""
    rng = np.random.Generator(np.random.PCG64(4242 + seed))
    rows = (np.arange(ENV_ROWS) + 0.5) / ENV_ROWS            # 0 at +z
    sky = np.where(rows < 0.5, 1.0 - rows, 0.15)[:, None, None] * np.array([0.8, 0.9, 1.2])[None, None]
    env = sky * np.ones((ENV_ROWS, ENV_COLS, 3)) + rng.uniform(0.0, 0.2, (ENV_ROWS, ENV_COLS, 3))
    r, c = rng.integers(1, 6), rng.integers(0, ENV_COLS)
    env[r, c] = [20.0, 18.0, 15.0]
    return env.astype(np.float32)


def make_visibility(n: int, K: int, seed: int = 0) -> np.ndarray:
    """[n, K] visibility values in [0, 1], a quarter exactly 1 and a tenth exactly 0 (float32)."""
    rng = np.random.Generator(np.random.PCG64(777 + seed))
    v = rng.uniform(0.0, 1.0, (n, K))
    u = rng.uniform(0.0, 1.0, (n, K))
    v[u < 0.25] = 1.0
    v[u > 0.9] = 0.0
    return v.astype(np.float32)


CAMERA = np.array([3.0, -2.5, 2.8], np.float32)
