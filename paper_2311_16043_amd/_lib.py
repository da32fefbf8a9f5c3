"""ctypes binding of librvis.so (argument marshalling only).

The library must have been built (`python -m paper_2311_16043_amd.build` or
`__graft_entry__.build()`); there is no fallback of any kind: if the shared
object is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librvis.so")

RV_OK = 0
RV_ERR_INVALID_ARG = -1
RV_ERR_WORKSPACE = -2
RV_ERR_HIP = -3
RV_ERR_UNSUPPORTED = -4
RV_MAX_GAUSSIANS = 1 << 30


class RvGaussians(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity", C.c_void_p), ("normal", C.c_void_p), ("n", C.c_int64)]


class RvTraceParams(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("T_min", C.c_float),
                ("sigma_cut", C.c_float), ("tmin_scale", C.c_float), ("dir_mode", C.c_int32)]


class RvBvhArrays(C.Structure):
    _fields_ = [("n", C.c_int64), ("header", C.c_void_p), ("keys", C.c_void_p), ("perm", C.c_void_p),
                ("nodes", C.c_void_p), ("parent", C.c_void_p), ("leaf_records", C.c_void_p),
                ("leaf_boxes", C.c_void_p), ("origins", C.c_void_p), ("nodes4", C.c_void_p)]


class RvTrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("lr_min", C.c_float), ("seed", C.c_uint64),
                ("step0", C.c_int64), ("total_steps", C.c_int64)]


class RvSurrogateArrays(C.Structure):
    _fields_ = [("header", C.c_void_p), ("master", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("packed", C.c_void_p)]


class RvPbrMaterial(C.Structure):
    _fields_ = [("albedo", C.c_void_p), ("roughness", C.c_void_p), ("sh", C.c_void_p), ("env", C.c_void_p),
                ("camera", C.c_float * 3), ("f0", C.c_float)]


class RvError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_vp, _i64, _i32, _f, _sz = C.c_void_p, C.c_int64, C.c_int32, C.c_float, C.c_size_t
_PG = C.POINTER(RvGaussians)
_PP = C.POINTER(RvTraceParams)

# name -> (restype, argtypes)
SIGNATURES = {
    "rv_last_error": (C.c_char_p, []),
    "rv_version": (C.c_char_p, []),
    "rv_bvh_bytes": (_sz, [_i64]),
    "rv_build_workspace_bytes": (_sz, [_i64]),
    "rv_build_bvh": (_i32, [_PG, _vp, _sz, _vp, _sz, _vp]),
    "rv_refit_bvh": (_i32, [_PG, _vp, _sz, _vp, _sz, _vp]),
    "rv_bvh_view": (_i32, [_vp, _i64, C.POINTER(RvBvhArrays)]),
    "rv_trace_workspace_bytes": (_sz, [_i64, _i32]),
    "rv_trace_visibility": (_i32, [_vp, _PG, _vp, _i32, _PP, _vp, _vp, _vp, _sz, _vp]),
    "rv_trace_rays": (_i32, [_vp, _PG, _vp, _i32, _PP, _vp, _i64, _vp, _vp]),
    "rv_trace_stats": (_i32, [_vp, _PG, _vp, _i32, _PP, _vp, _vp, _sz, _vp]),
    "rv_trace_visibility_backward": (_i32, [_vp, _PG, _vp, _i32, _PP, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rv_stream_copy": (_i32, [_vp, _vp, _sz, _vp]),
    "rv_gather_probe": (_i32, [_vp, _i64, _i32, _i32, _vp, _vp]),
    "rv_stream_read_sink_words": (_sz, [_sz]),
    "rv_stream_read": (_i32, [_vp, _sz, _vp, _vp]),
    "rv_trace_static_scratch_bytes": (_sz, []),
    "rv_trace_visibility_static": (_i32, [_vp, _PG, _vp, _i32, _PP, _vp, _vp, _vp]),
    "rv_surrogate_n_params": (_i64, []),
    "rv_surrogate_bytes": (_sz, []),
    "rv_surrogate_view": (_i32, [_vp, C.POINTER(RvSurrogateArrays)]),
    "rv_surrogate_train_workspace_bytes": (_sz, [_i32]),
    "rv_surrogate_infer_workspace_bytes": (_sz, [_i64]),
    "rv_surrogate_init": (_i32, [_vp, C.c_uint64, _vp, _vp, _vp, _vp]),
    "rv_surrogate_loss_grad": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "rv_surrogate_train": (_i32, [_vp, _vp, _vp, _vp, _i64, C.POINTER(RvTrainOpts), _vp, _vp, _sz, _vp]),
    "rv_surrogate_infer_xd": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "rv_surrogate_infer": (_i32, [_vp, _vp, _PG, _vp, _i32, _PP, _i64, _i64, _f, _vp, _vp, _vp, _vp, _sz,
                                  _vp]),
    "rv_ray_setup": (_i32, [_PG, _vp, _i32, _PP, _vp, _i64, _vp, _vp, _vp]),
    "rv_trace_sh_workspace_bytes": (_sz, [_i64, _i32]),
    "rv_trace_visibility_sh": (_i32, [_vp, _PG, _vp, _i32, _PP, _vp, _vp, _vp, _sz, _vp]),
    "rv_shade_pbr": (_i32, [_PG, _vp, _i32, _PP, _vp, C.POINTER(RvPbrMaterial), _vp, _vp]),
}

_lib = None


def load() -> C.CDLL:
    """Load librvis.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           f"(python -m paper_2311_16043_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().rv_last_error().decode()


def check(fn: str, status: int) -> None:
    if status != RV_OK:
        raise RvError(fn, status, last_error())


def call(fn: str, *args) -> None:
    check(fn, getattr(load(), fn)(*args))
