"""ctypes binding of libtetsplat.so (include/tetsplat.h).  Marshalling only:
every step of the rendering runs in the HIP kernels behind this ABI."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtetsplat.so")

RENDER_OK, RENDER_EINVAL, RENDER_ENOSPC, RENDER_EHIP, RENDER_EOVERFLOW = 0, -1, -2, -3, -4
RENDER_RECOMPUTE_STATE, RENDER_VALIDATE, RENDER_DETERMINISTIC, RENDER_RECORD_GRADS = 1, 2, 4, 8
RENDER_WINDOW_MAX = 8


class render_scene(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("tets", C.c_void_p), ("sdf", C.c_void_p), ("colors", C.c_void_p),
                ("V", C.c_int32), ("K", C.c_int32), ("s", C.c_float)]


class render_view(C.Structure):
    _fields_ = [("scene", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("R", C.c_float * 9),
                ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("znear", C.c_float), ("bg", C.c_float * 3), ("out", C.c_void_p)]


class render_params(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("flags", C.c_int32), ("waves", C.c_int32),
                ("alpha_min", C.c_float),
                ("alpha_clamp", C.c_float), ("t_min", C.c_float), ("prefilter_tf", C.c_float),
                ("window", C.c_int32), ("chunk_fwd", C.c_int32), ("chunk_bwd", C.c_int32)]


class render_grads(C.Structure):
    _fields_ = [("dverts", C.c_void_p), ("dsdf", C.c_void_p), ("dcolors", C.c_void_p)]


class render_status(C.Structure):
    _fields_ = [("entries", C.c_int64), ("kept", C.c_int64), ("records", C.c_int64), ("overflow", C.c_int32),
                ("invalid_index", C.c_int32), ("entry_capacity", C.c_int64), ("kept_capacity", C.c_int64),
                ("entries_needed", C.c_int64)]


class render_debug_view(C.Structure):
    _fields_ = [("tile_keys", C.c_void_p), ("entry_record", C.c_void_p), ("kept_tet", C.c_void_p),
                ("view_rec_base", C.c_void_p), ("scene_kept_base", C.c_void_p), ("scene_kept_count", C.c_void_p),
                ("ranges", C.c_void_p), ("last", C.c_void_p), ("t_last", C.c_void_p),
                ("total_tiles", C.c_int64), ("total_pixels", C.c_int64)]


class RenderError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"render error {code}: {msg}")
        self.code = code


_lib = None

EXPORTS = ("render_workspace_size", "render_forward", "render_backward", "render_read_status",
           "render_debug_pointers", "render_last_error", "render_profile", "render_profile_read",
           "render_decode_status", "render_mesh_edges_workspace_size", "render_mesh_edges",
           "render_regularizers_workspace_size", "render_regularizers", "render_marching_tets_workspace_size",
           "render_marching_tets", "render_prefilter_bounds", "render_cube_grid", "render_refit_cube",
           "render_forward_static")
STATIC_WORKSPACE_BYTES = 64 << 20
STATUS_BYTES = 256

STAGES = ("upload", "prefilter", "project", "depth_sort", "scan", "emit", "pair_grads", "ranges", "composite",
          "zero_grads", "composite_bwd", "vertex_bwd")


def lib():
    """Load the in-tree HIP library.  There is no fallback: a missing or
    unloadable library is an error."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2406_01579_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I, I64 = C.c_void_p, C.c_int, C.c_int64
        L.render_workspace_size.argtypes = [P, I, P, I, P, I64, I64, C.POINTER(C.c_size_t)]
        L.render_forward.argtypes = [P, I, P, I, P, I64, I64, P, C.c_size_t, P]
        L.render_forward_static.argtypes = [P, I, P, I, P, I64, I64, P, P]
        L.render_backward.argtypes = [P, I, P, I, P, I64, I64, P, C.c_size_t, P, P, P]
        L.render_read_status.argtypes = [P, P, P]
        L.render_debug_pointers.argtypes = [P, I, P, I, P, I64, I64, P, P]
        L.render_last_error.restype = C.c_char_p
        L.render_profile.argtypes = [I]
        L.render_profile_read.argtypes = [P, P]
        L.render_decode_status.argtypes = [P, P]
        I32 = C.c_int32
        L.render_mesh_edges_workspace_size.argtypes = [I32, C.POINTER(C.c_size_t)]
        L.render_mesh_edges.argtypes = [P, I32, I32, P, P, P, C.c_size_t, P]
        L.render_regularizers_workspace_size.argtypes = [I32, I32, C.POINTER(C.c_size_t)]
        L.render_regularizers.argtypes = [P, P, P, I32, I32, P, P, I64, P, P, P, P, P, C.c_size_t, P]
        L.render_prefilter_bounds.argtypes = [P, P, P, P, P]
        L.render_cube_grid.argtypes = [I32, P, P, P, P]
        L.render_refit_cube.argtypes = [P, P, I32, P, P]
        L.render_marching_tets_workspace_size.argtypes = [I32, I64, C.POINTER(C.c_size_t)]
        L.render_marching_tets.argtypes = [P, P, P, I32, I32, P, P, I64, P, I64, P, I64, P, P, C.c_size_t, P]
        for name in EXPORTS:
            getattr(L, name)
        _lib = L
    return _lib


def check(rc: int):
    if rc != RENDER_OK:
        raise RenderError(rc, lib().render_last_error().decode())
    return rc


def profile(enable: bool):
    check(lib().render_profile(1 if enable else 0))


def profile_read() -> dict:
    """{stage: (total_ms, launches)} accumulated since profile(True)."""
    ms = (C.c_double * len(STAGES))()
    cnt = (C.c_int64 * len(STAGES))()
    check(lib().render_profile_read(ms, cnt))
    return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}
