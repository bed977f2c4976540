"""Particle generation front end (sections 3.1.1-3.2.1) through
fppg_generate: background-grid cell classes and the initial volume and
surface particles of a closed mesh, on the GPU."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import check, ptr
from .relax import Context


def generate(vert, tri, dx: float, origin, dims, device: int = 0, ctx: Context | None = None, cap: int | None = None):
    """Classify the cells of the grid (origin, dx, dims = (nx, ny, nz)) and seed
    particles. Returns (cls uint8 [nz, ny, nx] with 0 external / 1 internal /
    2 surface, pos float32 [P, 4] with the tag bits in w, owner int32 [P]:
    the facet of a surface particle, -1 for a volume particle), particles in
    cell order."""
    if not torch.cuda.is_available():
        raise RuntimeError("generate() needs a GPU (no CPU fallback)")
    ctx = ctx or Context(device)
    dev = torch.device("cuda", device)
    vert = np.ascontiguousarray(vert, np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
    nx, ny, nz = (int(v) for v in dims)
    cls = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    if cap is None:
        cap = nx * ny * nz
    pos = torch.empty((max(cap, 1), 4), dtype=torch.float32, device=dev)
    owner = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    d = (ctypes.c_int32 * 3)(nx, ny, nz)
    counts = (ctypes.c_int64 * 2)()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    check(ctx.lib.fppg_generate(ctx.handle, vert.ctypes.data_as(ctypes.c_void_p), len(vert),
                                tri.ctypes.data_as(ctypes.c_void_p), len(tri), float(dx), o, d, ptr(cls),
                                ptr(pos), ptr(owner), int(cap), counts, stream), ctx.handle)
    n = int(counts[0]) + int(counts[1])
    return cls, pos[:n], owner[:n]


def generate_sparse(vert, tri, dx: float, origin, dims, device: int = 0, ctx: Context | None = None,
                    cap: int | None = None):
    """The particles of generate() through the sparse cell storage (no dense
    class array; fppg_generate_sparse). Returns (pos float32 [P, 4], owner
    int32 [P], stats dict: registered cells, crossing events, events after
    cancellation, subdivision levels). Without cap, a first call sizes the
    output."""
    if not torch.cuda.is_available():
        raise RuntimeError("generate_sparse() needs a GPU (no CPU fallback)")
    ctx = ctx or Context(device)
    dev = torch.device("cuda", device)
    vert = np.ascontiguousarray(vert, np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    counts = (ctypes.c_int64 * 2)()
    stats = (ctypes.c_int64 * 4)()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

    def call(cap_, pos, owner):
        return ctx.lib.fppg_generate_sparse(ctx.handle, vert.ctypes.data_as(ctypes.c_void_p), len(vert),
                                            tri.ctypes.data_as(ctypes.c_void_p), len(tri), float(dx), o, d,
                                            ptr(pos), ptr(owner), int(cap_), counts, stats, stream)

    pos = torch.empty((max(cap or 1, 1), 4), dtype=torch.float32, device=dev)
    owner = torch.empty(max(cap or 1, 1), dtype=torch.int32, device=dev)
    rc = call(cap or 0, pos, owner)
    if rc == L.E_CAPACITY and cap is None and counts[0] == -1:
        n = int(counts[1])
        pos = torch.empty((max(n, 1), 4), dtype=torch.float32, device=dev)
        owner = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        rc = call(n, pos, owner)
    check(rc, ctx.handle)
    n = int(counts[0]) + int(counts[1])
    info = {"cells": int(stats[0]), "events": int(stats[1]), "toggles": int(stats[2]), "levels": int(stats[3])}
    return pos[:n], owner[:n], info


def features(vert, tri, cos_threshold: float, dx: float, device: int = 0, ctx: Context | None = None):
    """Feature edges, singular vertices, feature lines and feature-line
    particles of a mesh (fppg_features). Returns a dict of device tensors:
    edges [E, 2], singular [S], line_begin [L + 1], line_vert [V],
    line_closed [L], pos [P, 4] (w = tag bits), line_of [P], arc [P] (float64),
    seg [P] (segment of the line) and u [P] (float64, arc length inside it)."""
    if not torch.cuda.is_available():
        raise RuntimeError("features() needs a GPU (no CPU fallback)")
    ctx = ctx or Context(device)
    dev = torch.device("cuda", device)
    vert = np.ascontiguousarray(vert, np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

    def call(o):
        return ctx.lib.fppg_features(ctx.handle, vert.ctypes.data_as(ctypes.c_void_p), len(vert),
                                     tri.ctypes.data_as(ctypes.c_void_p), len(tri), float(cos_threshold), float(dx),
                                     ctypes.byref(o), stream)

    sizes = L.FeaturesOut()
    check(call(sizes), ctx.handle)   # line_begin = NULL: sizes only
    t = {"edges": torch.empty((max(sizes.n_edges, 1), 2), dtype=torch.int32, device=dev),
         "singular": torch.empty(max(sizes.n_singular, 1), dtype=torch.int32, device=dev),
         "line_begin": torch.empty(sizes.n_lines + 1, dtype=torch.int32, device=dev),
         "line_vert": torch.empty(max(sizes.n_line_vert, 1), dtype=torch.int32, device=dev),
         "line_closed": torch.empty(max(sizes.n_lines, 1), dtype=torch.uint8, device=dev),
         "pos": torch.empty((max(sizes.n_particles, 1), 4), dtype=torch.float32, device=dev),
         "line_of": torch.empty(max(sizes.n_particles, 1), dtype=torch.int32, device=dev),
         "arc": torch.empty(max(sizes.n_particles, 1), dtype=torch.float64, device=dev),
         "seg": torch.empty(max(sizes.n_particles, 1), dtype=torch.int32, device=dev),
         "u": torch.empty(max(sizes.n_particles, 1), dtype=torch.float64, device=dev)}
    o = L.FeaturesOut(ptr(t["edges"]), sizes.n_edges, ptr(t["singular"]), sizes.n_singular, ptr(t["line_begin"]),
                      ptr(t["line_vert"]), ptr(t["line_closed"]), sizes.n_lines, sizes.n_line_vert, ptr(t["pos"]),
                      ptr(t["line_of"]), ptr(t["arc"]), ptr(t["seg"]), ptr(t["u"]), sizes.n_particles)
    check(call(o), ctx.handle)
    n = {"edges": o.n_edges, "singular": o.n_singular, "line_vert": o.n_line_vert, "line_closed": o.n_lines,
         "pos": o.n_particles, "line_of": o.n_particles, "arc": o.n_particles, "seg": o.n_particles,
         "u": o.n_particles}
    return {k: (v[: n[k]] if k in n else v) for k, v in t.items()}


UNION, INTERSECTION, DIFFERENCE = 0, 1, 2


def cells_boolean(cls_a: torch.Tensor, cls_b: torch.Tensor, op: int, ctx: Context | None = None) -> torch.Tensor:
    """Boolean combination (fppg_cells_boolean) of two class arrays of generate()
    on the same grid: op UNION, INTERSECTION or DIFFERENCE (a - b)."""
    if cls_a.shape != cls_b.shape or cls_a.dtype != torch.uint8 or cls_b.dtype != torch.uint8:
        raise ValueError("class arrays of the same grid (uint8) expected")
    ctx = ctx or Context(cls_a.device.index or 0)
    a, b = cls_a.contiguous(), cls_b.contiguous()
    out = torch.empty_like(a)
    stream = ctypes.c_void_p(torch.cuda.current_stream(a.device).cuda_stream)
    check(ctx.lib.fppg_cells_boolean(ctx.handle, ptr(a), ptr(b), a.numel(), int(op), ptr(out), stream), ctx.handle)
    return out


class SparseGrid:
    """The sparse storage of the cells a mesh meets (fppg_sparse_grid_*):
    facet subdivision and registration on the grid (origin, cell, dims =
    (nx, ny, nz)), C_compact in Morton order and the hash table of Eq. 10."""

    def __init__(self, vert, tri, origin, cell: float, dims, pad: float = 0.0, hash_size: int = 0,
                 device: int = 0, ctx: Context | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("SparseGrid needs a GPU (no CPU fallback)")
        self.ctx = ctx or Context(device)
        self.dev = torch.device("cuda", device)
        vert = np.ascontiguousarray(vert, np.float64).reshape(-1, 3)
        tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
        o = (ctypes.c_double * 3)(*[float(v) for v in origin])
        d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
        h = ctypes.c_void_p()
        check(self.ctx.lib.fppg_sparse_grid_create(self.ctx.handle, vert.ctypes.data_as(ctypes.c_void_p), len(vert),
                                                   tri.ctypes.data_as(ctypes.c_void_p), len(tri), o, float(cell), d,
                                                   float(pad), int(hash_size), ctypes.byref(h)), self.ctx.handle)
        self.handle = h
        v = L.SparseGridView()
        check(self.ctx.lib.fppg_sparse_grid_info(self.handle, ctypes.byref(v)), self.ctx.handle)
        self.n_entry, self.n_cell, self.hash_size, self.levels = v.n_entry, v.n_cell, v.hash_size, v.levels

    def arrays(self) -> dict:
        """Device copies of the structure's arrays."""
        def e(n, dt):
            return torch.empty(max(int(n), 1), dtype=dt, device=self.dev)
        t = {"facets": e(self.n_entry, torch.int32), "morton": e(self.n_cell, torch.int64),
             "begin": e(self.n_cell, torch.int32), "length": e(self.n_cell, torch.int32),
             "order": e(self.n_cell, torch.int32), "h_begin": e(self.hash_size + 1, torch.int32),
             "h_length": e(self.hash_size, torch.int32)}
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)
        check(self.ctx.lib.fppg_sparse_grid_copy(self.ctx.handle, self.handle, *[ptr(t[k]) for k in
                                                 ("facets", "morton", "begin", "length", "order", "h_begin",
                                                  "h_length")], stream), self.ctx.handle)
        n = {"facets": self.n_entry, "morton": self.n_cell, "begin": self.n_cell, "length": self.n_cell,
             "order": self.n_cell, "h_begin": self.hash_size + 1, "h_length": self.hash_size}
        return {k: v[: int(n[k])] for k, v in t.items()}

    def lookup(self, points: torch.Tensor):
        """(begin, length) [P] of the facets of each point's cell (-1, 0: none)."""
        p = points.to(self.dev, torch.float64).contiguous()
        n = p.shape[0]
        b = torch.empty(max(n, 1), dtype=torch.int32, device=self.dev)
        ln = torch.empty(max(n, 1), dtype=torch.int32, device=self.dev)
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)
        check(self.ctx.lib.fppg_sparse_grid_lookup(self.ctx.handle, self.handle, n, ptr(p), ptr(b), ptr(ln), stream),
              self.ctx.handle)
        return b[:n], ln[:n]

    def close(self):
        if self.handle:
            self.ctx.lib.fppg_sparse_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
