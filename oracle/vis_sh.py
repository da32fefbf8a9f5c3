"""FP64 reference of visibility compressed to spherical harmonics. TEST
INFRASTRUCTURE ONLY: tests, smoke() and the CPU baseline of bench.py use it.

Each Gaussian's visibility over its K directions (Sec. 4.2) is projected onto
the real spherical harmonics of degree <= 2 -- the "3-level SH" the paper uses
for the indirect light (Sec. 3.3) -- by the same quadrature as Eq. (10):

    v_ij = sum_k V_ik Y_j(d_k) dw,   dw = 2 pi / K (hemisphere), 4 pi / K (sphere),

with d_k the unit directions of the table in the frame the rays use: the
local frame about the normal (z = n) in hemisphere mode, the world frame in
sphere mode. V(w) ~ sum_j v_ij Y_j(w_local) then reconstructs the visibility
from 9 numbers instead of K.
"""
from __future__ import annotations

import math

import numpy as np

from .pbr import sh_basis

N_SH = 9


def weights(dirs, dir_mode: int) -> np.ndarray:
    """[K, 9] projection weights Y_j(d_k) dw of the direction table."""
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    dw = (2.0 if dir_mode == 1 else 4.0) * math.pi / d.shape[0]
    return sh_basis(d) * dw


def project(vis, dirs, dir_mode: int) -> np.ndarray:
    """[n, 9] SH coefficients of the visibility vis [n, K]."""
    return np.asarray(vis, np.float64) @ weights(dirs, dir_mode)


def project_bounds(v_lo, v_hi, dirs, dir_mode: int):
    """Interval of the projection when each V_ik is only known to lie in
    [v_lo, v_hi] (elementwise): ([n, 9] low, [n, 9] high)."""
    W = weights(dirs, dir_mode)
    lo = np.asarray(v_lo, np.float64)
    hi = np.asarray(v_hi, np.float64)
    Wp, Wn = np.maximum(W, 0.0), np.minimum(W, 0.0)
    return lo @ Wp + hi @ Wn, hi @ Wp + lo @ Wn
