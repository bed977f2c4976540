"""ctypes binding of libfppg.so: the entry points of include/fppg.h with the same names.

Argument marshalling only. The library is built in-tree by build.py; loading
fails loudly when it is missing or does not export the declared entry points.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint8, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfppg.so")

OK, E_ARG, E_HIP, E_WORKSPACE, E_CAPACITY, E_UNSUPPORTED, E_NODEVICE = 0, -1, -2, -3, -4, -5, -6
F_COUNT_PAIRS = 1
F_FORCES_ONLY = 2   # fppg_relax_step: accel and amax only, no displacement
CSG_NONE, CSG_UNION, CSG_DIFFERENCE = 0, 1, 2
S_NONFINITE_ACCEL, S_NONFINITE_POS, S_BAD_INDEX, S_FIXED_RANGE = 1, 2, 4, 8
C_REVERT_SURFACE, C_REVERT_FEATURE, C_REVERT_VOLUME = 0, 1, 2
NCOUNTERS = 8
NPHASES = 5
PHASES = ("build_cells", "force", "update", "project", "hvp")


class GeomDesc(ctypes.Structure):
    _fields_ = [
        ("origin", c_float * 3), ("inv_cell", c_float), ("dims", c_int32 * 3), ("k", c_int32),
        ("h", c_float), ("proj_radius", c_float), ("part_begin", c_int64), ("part_end", c_int64),
        ("vert", POINTER(c_double)), ("n_vert", c_int32),
        ("tri", POINTER(c_int32)), ("n_tri", c_int32),
        ("line_seg_begin", POINTER(c_int32)), ("n_line", c_int32),
        ("seg_p", POINTER(c_double)), ("line_closed", POINTER(c_uint8)),
        ("seg_vert", POINTER(c_int32)),
        ("slab", c_int32),
        ("csg_op", c_int32), ("n_part", c_int32), ("part_tri_begin", POINTER(c_int32)),
        ("max_level", c_int32),
    ]


_P = c_void_p
_SIGS = {
    "fppg_create": (c_int32, [c_int32, POINTER(c_void_p)]),
    "fppg_destroy": (None, [_P]),
    "fppg_status_str": (c_char_p, [c_int32]),
    "fppg_last_error": (c_char_p, [_P]),
    "fppg_read_status": (c_int32, [_P, _P, POINTER(c_uint32)]),
    "fppg_profile": (c_int32, [_P, c_uint32]),
    "fppg_profile_read": (c_int32, [_P, POINTER(c_double), POINTER(c_int64)]),
    "fppg_geom_create": (c_int32, [_P, POINTER(GeomDesc), c_int32, POINTER(c_void_p)]),
    "fppg_geom_destroy": (None, [_P]),
    "fppg_geom_info": (c_int32, [_P, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64),
                                 POINTER(c_int64), POINTER(c_int64)]),
    "fppg_workspace_size": (c_int32, [_P, c_int64, POINTER(c_size_t)]),
    "fppg_geom_search_grid": (c_int32, [_P, _P, _P, _P, _P, _P]),
    "fppg_build_cells": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, _P, _P, _P, _P, c_size_t, _P]),
    "fppg_relax_step": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, c_int32, c_uint32, c_uint32,
                                  _P, _P, _P, _P, c_int32, _P, c_size_t, _P]),
    "fppg_project": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, _P, c_int32, c_uint32, _P, _P, c_int32, _P,
                               c_size_t, _P]),
    "fppg_moving_list": (c_int32, [_P, _P, c_int64, _P, c_uint32, _P, _P, _P, c_size_t, _P]),
    "fppg_set_launch": (c_int32, [_P, c_int32, c_int32]),
    "fppg_set_schedule": (c_int32, [_P, c_int32]),
    "fppg_tier_partition": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, _P, _P, c_uint32, _P, _P, c_size_t, _P]),
    "fppg_volume_layers": (c_int32, [_P, _P, c_int64, _P, c_double, _P, _P]),
    "fppg_generate": (c_int32, [_P, _P, c_int32, _P, c_int32, c_double, _P, _P, _P, _P, _P, c_int64, _P, _P]),
    "fppg_generate_sparse": (c_int32, [_P, _P, c_int32, _P, c_int32, c_double, _P, _P, _P, _P, c_int64, _P, _P,
                                       _P]),
    "fppg_features": (c_int32, [_P, _P, c_int32, _P, c_int32, c_double, c_double, _P, _P]),
    "fppg_cells_boolean": (c_int32, [_P, _P, _P, c_int64, c_int32, _P, _P]),
    "fppg_relax_hvp": (c_int32, [_P, _P, c_int64, _P, _P, c_uint32, c_int32, _P, _P, _P]),
    "fppg_debug_neighbors": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, c_int32, _P]),
    "fppg_graph_create": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, c_int32, c_uint32,
                                    _P, _P, _P, _P, c_size_t, c_int32, _P, POINTER(c_void_p)]),
    "fppg_graph_launch": (c_int32, [_P, _P, c_int32, _P]),
    "fppg_graph_destroy": (None, [_P]),
    "fppg_relax_energy": (c_int32, [_P, _P, c_int64, _P, _P, c_uint32, _P, _P, c_size_t, _P]),
    "fppg_vec_dot": (c_int32, [_P, c_int64, _P, _P, _P, _P, c_size_t, _P]),
    "fppg_vec_dot_noalloc": (c_int32, [_P, c_int64, _P, _P, _P, _P]),
    "fppg_vec_axpby": (c_int32, [_P, c_int64, c_float, _P, c_float, _P, _P]),
    "fppg_vec_maxnorm": (c_int32, [_P, c_int64, _P, _P, _P]),
    "fppg_vec_clamp": (c_int32, [_P, c_int64, _P, c_float, _P]),
    "fppg_tangent_project": (c_int32, [_P, _P, c_int64, _P, _P, _P, c_int32, c_uint32, _P, _P]),
    "fppg_displace": (c_int32, [_P, _P, c_int64, _P, _P, _P, c_int32, c_uint32, _P, c_float, _P, _P]),
    "fppg_project_record": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, _P, c_int32, c_uint32, _P, _P, _P,
                                      c_size_t, _P]),
    "fppg_uniformity_loss": (c_int32, [_P, _P, c_int64, _P, _P, c_uint32, c_double, _P, _P, _P, c_size_t, _P]),
    "fppg_step_adjoint": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, c_int32, c_uint32,
                                    _P, _P, _P, _P, _P]),
    "fppg_fixed_adjoint": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, c_int32, c_uint32, _P, _P, _P]),
    "fppg_vec_permute": (c_int32, [_P, c_int64, _P, _P, c_int32, _P, _P]),
    "fppg_vec_combine3": (c_int32, [_P, c_int64, c_float, _P, c_float, _P, c_float, _P, _P, c_float, _P, _P]),
    "fppg_relax_hvp_projected": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P, c_int32, c_uint32, _P, c_float, _P,
                                           _P]),
    "fppg_fixed_to_double": (c_int32, [_P, c_int64, _P, _P, _P]),
    "fppg_lattice_density": (c_int32, [c_double, c_double, POINTER(c_double)]),
    "fppg_source_hash": (c_char_p, []),
    "fppg_sparse_grid_create": (c_int32, [_P, _P, c_int32, _P, c_int32, POINTER(c_double), c_double,
                                          POINTER(c_int32), c_double, c_int64, POINTER(c_void_p)]),
    "fppg_sparse_grid_info": (c_int32, [_P, _P]),
    "fppg_sparse_grid_copy": (c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "fppg_sparse_grid_lookup": (c_int32, [_P, _P, c_int64, _P, _P, _P, _P]),
    "fppg_sparse_grid_destroy": (c_int32, [_P]),
}

_lib = None


class FeaturesOut(ctypes.Structure):
    """fppg_features_out."""
    _fields_ = [
        ("edges", c_void_p), ("cap_edges", c_int64), ("singular", c_void_p), ("cap_singular", c_int64),
        ("line_begin", c_void_p), ("line_vert", c_void_p), ("line_closed", c_void_p),
        ("cap_lines", c_int64), ("cap_line_vert", c_int64),
        ("pos", c_void_p), ("line_of", c_void_p), ("arc", c_void_p), ("seg", c_void_p), ("u", c_void_p),
        ("cap_particles", c_int64),
        ("n_edges", c_int64), ("n_singular", c_int64), ("n_lines", c_int64), ("n_line_vert", c_int64),
        ("n_particles", c_int64),
    ]


class SparseGridView(ctypes.Structure):
    """fppg_sparse_grid_view."""
    _fields_ = [
        ("n_entry", c_int64), ("n_cell", c_int64), ("hash_size", c_int64), ("levels", c_int64),
        ("facets", c_void_p), ("morton", c_void_p), ("begin", c_void_p), ("length", c_void_p),
        ("order", c_void_p), ("h_begin", c_void_p), ("h_length", c_void_p),
    ]


class FppgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fppg status {status}: {msg}")
        self.status = status


def lib():
    """Load libfppg.so. A library that is missing, or whose embedded source
    hash differs from the sources in the tree (a stale build), is rebuilt
    first; if that fails the import fails loudly."""
    global _lib
    if _lib is not None:
        return _lib
    from . import build as B
    want = B.source_hash()
    if B.built_hash(LIB_PATH) != want:
        B.build()
        if B.built_hash(LIB_PATH) != want:
            raise RuntimeError(f"{LIB_PATH}: the rebuilt library does not carry the source hash {want}")
    L = ctypes.CDLL(LIB_PATH)
    got = L.fppg_source_hash
    got.restype = c_char_p
    got.argtypes = []
    if got().decode() != want:
        raise RuntimeError(f"{LIB_PATH} reports source hash {got().decode()}, the sources have {want}")
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)        # AttributeError = library does not export it: fail loudly
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status, ctx=None):
    if status != OK:
        L = lib()
        msg = L.fppg_last_error(ctx).decode() if ctx else L.fppg_status_str(status).decode()
        raise FppgError(status, msg or L.fppg_status_str(status).decode())
    return status


def ptr(t):
    """Device (or host) address of a torch tensor / numpy array, or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return c_void_p(t.data_ptr())
    return c_void_p(t.ctypes.data)
