"""Shared helpers of the GPU parity tests (oracle side and comparison only)."""
from __future__ import annotations

import numpy as np

import oracle

TOL = 1e-4  # absolute visibility tolerance in FP32 against the FP64 oracle


def oracle_lbvh(scene: dict) -> dict:
    lo, hi, keys = oracle.morton63(scene["mean"])
    order = oracle.sort_keys(keys)
    tree = oracle.radix_tree(keys[order])
    return dict(lo=lo, hi=hi, keys=keys, order=order, **tree)


def check_vis(v_gpu: np.ndarray, orc: dict, tol: float = TOL, label: str = "") -> dict:
    """GPU visibility must lie in [V_lo - tol, V_hi + tol]; for rays with no
    ambiguous Gaussian this is |V_gpu - P| <= tol."""
    v = np.asarray(v_gpu, dtype=np.float64)
    lo = orc["V_lo"] - tol
    hi = orc["V_hi"] + tol
    bad = ~((v >= lo) & (v <= hi))
    err = np.abs(v - orc["P"])
    clean = orc["n_amb"] == 0
    # ambiguous rays whose value is not the plain definition's: binary32 took
    # the other decision on at least one pair within rounding of a cut
    non_p = int(((~clean) & (err > tol)).sum())
    stats = dict(rays=int(v.size), ambiguous_rays=int((~clean).sum()), ambiguous_non_p=non_p, fails=int(bad.sum()),
                 max_err_clean=float(err[clean].max()) if clean.any() else 0.0,
                 mean_err=float(err.mean()), max_err=float(err.max()))
    print(f"[parity {label}] {stats}", flush=True)
    if bad.any():
        idx = np.nonzero(bad)[0][:10]
        detail = [(int(i), float(v[i]), float(orc["P"][i]), float(orc["V_lo"][i]), float(orc["V_hi"][i]))
                  for i in idx]
        raise AssertionError(f"{label}: {int(bad.sum())} rays outside the acceptance band: {detail}")
    return stats
