"""ctypes binding of libfr.so (the C ABI declared in include/fr.h).

Argument marshalling only: every step of the render runs in the HIP library.
The library must have been built (paper_2101_05356_amd/build.py); if it is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfr.so")

FR_OK, FR_ERR_INVALID_ARG, FR_ERR_SHAPE, FR_ERR_OOM, FR_ERR_BUDGET = 0, 1, 2, 3, 4
FR_ERR_DEVICE, FR_ERR_NONFINITE, FR_ERR_LIMIT, FR_ERR_NOT_FOUND = 5, 6, 7, 8
FR_REFIT, FR_REBUILD = 0, 1
FR_BRDF_PRINTED, FR_BRDF_NORMALIZED = 0, 1

P = ctypes.c_void_p


class FrScene(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("n_lights", ctypes.c_int32),
                ("verts", P), ("diffuse", P), ("specular", P), ("roughness", P),
                ("light_p0", P), ("light_e1", P), ("light_e2", P), ("light_rad", P), ("light_shape", P),
                ("cam", P), ("fov_y", ctypes.c_float), ("step", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class FrRenderOpts(ctypes.Structure):
    _fields_ = [("brdf_variant", ctypes.c_int32), ("components", ctypes.c_int32),
                ("edge_samples", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dbg_hit", P), ("dbg_pflag", P), ("dbg_vis", P), ("dbg_stats", P)]


class FrGrads(ctypes.Structure):
    _fields_ = [("verts", P), ("normals", P), ("diffuse", P), ("specular", P), ("roughness", P),
                ("light_geom", P), ("light_rad", P), ("cam", P)]


class FrError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FrError(f"HIP library {LIB_PATH} is not built: run paper_2101_05356_amd/build.py "
                      "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    i32, u64 = ctypes.c_int32, ctypes.c_uint64
    sig = {
        "fr_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "fr_last_error": ([P], ctypes.c_char_p),
        "fr_ctx_create": ([ctypes.c_int, P], ctypes.c_int),
        "fr_ctx_destroy": ([P], ctypes.c_int),
        "fr_mesh_create": ([P, i32, i32, P, P], ctypes.c_int),
        "fr_mesh_destroy": ([P], ctypes.c_int),
        "fr_mesh_update": ([P, P, ctypes.c_int, P], ctypes.c_int),
        "fr_mesh_normals": ([P], P),
        "fr_mesh_edges": ([P, P, P], i32),
        "fr_mesh_bvh_depth": ([P], i32),
        "fr_render_forward": ([P, P, P, P, P], ctypes.c_int),
        "fr_loss": ([P, P, i32, i32, i32, P, P, P], ctypes.c_int),
        "fr_render_backward": ([P, P, P, P, P, P], ctypes.c_int),
        "fr_blend": ([P, P, P, i32, i32, P, P], ctypes.c_int),
        "fr_blend_backward": ([P, P, i32, i32, P, P], ctypes.c_int),
        "fr_pose_forward": ([P, i32, P, P, P], ctypes.c_int),
        "fr_pose_backward": ([P, i32, P, P, P, P, P], ctypes.c_int),
        "fr_adam_step": ([P, P, P, P, P, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, P],
                         ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return _lib


def exported_symbols():
    """Names of the functions the binding expects the library to export."""
    return ["fr_status_string", "fr_last_error", "fr_ctx_create", "fr_ctx_destroy", "fr_mesh_create",
            "fr_mesh_destroy", "fr_mesh_update", "fr_mesh_normals", "fr_mesh_edges", "fr_mesh_bvh_depth",
            "fr_render_forward", "fr_loss", "fr_render_backward", "fr_blend", "fr_blend_backward",
            "fr_pose_forward", "fr_pose_backward", "fr_adam_step"]


def check(rc: int, ctx=None, what: str = ""):
    if rc != FR_OK:
        msg = lib().fr_status_string(rc).decode()
        if ctx:
            detail = lib().fr_last_error(ctx).decode()
            if detail:
                msg += f": {detail}"
        raise FrError(f"{what} failed ({rc}): {msg}")
