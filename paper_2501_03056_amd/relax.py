"""Python driver of the relaxation loop (Algorithm 1) on one GPU.

`Relaxer` owns the device state of a batch of geometries as torch tensors
(torch provides the device memory and the stream) and calls the four C-ABI
entry points in order every iteration:

    build_cells -> relax_step -> project

Particle state (structure of arrays, sorted by (cell, id) after build_cells):
    pos    float32 [N, 4]  x, y, z and the int32 bits tag | level << 3 | geometry << 8
    id     int32   [N]     original particle index
    owner  int32   [N]     facet (surface), feature slot (feature), else -1
    feat_seg int32 [F], feat_u float64 [F]  feature table (by slot, not permuted)
All arithmetic runs in the library's kernels; this module only marshals.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import check, ptr


def _pack_w(tag: np.ndarray, gid: np.ndarray, level: np.ndarray | None = None) -> np.ndarray:
    bits = (np.asarray(tag, np.int32) & 7) | (np.asarray(gid, np.int32) << 8)
    if level is not None:
        bits = bits | ((np.asarray(level, np.int32) & 3) << 3)
    return bits.astype(np.int32).view(np.float32)


def geom_descs(geoms):
    """ctypes descriptors of a batch; returns (array, keep-alive list)."""
    arr = (L.GeomDesc * len(geoms))()
    keep = []
    for g, geo in enumerate(geoms):
        d = arr[g]
        for q in range(3):
            d.origin[q] = float(geo.origin[q])
            d.dims[q] = int(geo.dims[q])
        d.inv_cell = float(geo.inv_cell)
        d.k = int(geo.k)
        d.h = float(geo.h)
        d.proj_radius = float(geo.proj_radius)
        d.max_level = int(getattr(geo, "max_level", 0))
        d.part_begin = int(geo.part_begin)
        d.part_end = int(geo.part_end)
        vert = np.ascontiguousarray(geo.mesh.vert, np.float64)
        tri = np.ascontiguousarray(geo.mesh.tri, np.int32)
        lines = geo.mesh.lines
        lsb = np.ascontiguousarray(lines.line_seg_begin, np.int32)
        segp = np.ascontiguousarray(lines.seg_p, np.float64).reshape(-1)
        closed = np.ascontiguousarray(lines.line_closed, np.uint8)
        keep += [vert, tri, lsb, segp, closed]
        d.vert = vert.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.n_vert = len(vert)
        d.tri = tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_tri = len(tri)
        d.line_seg_begin = lsb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_line = int(lines.n_line)
        d.seg_p = segp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(segp) else None
        d.line_closed = closed.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if len(closed) else None
        sv = getattr(lines, "seg_vert", None)
        if sv is not None and len(sv):
            sv = np.ascontiguousarray(sv, np.int32).reshape(-1)
            keep.append(sv)
            d.seg_vert = sv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        else:
            d.seg_vert = None
        d.slab = int(getattr(geo, "slab", 0))
        csg = getattr(geo, "csg", None)
        if csg is not None:
            tb = np.ascontiguousarray(csg.part_tri_begin, np.int32)
            keep.append(tb)
            d.csg_op = int(csg.op)
            d.n_part = len(tb) - 1
            d.part_tri_begin = tb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        else:
            d.csg_op, d.n_part, d.part_tri_begin = L.CSG_NONE, 0, None
    return arr, keep


class Context:
    """fppg_create / fppg_destroy."""

    def __init__(self, device: int = 0):
        self.lib = L.lib()
        h = ctypes.c_void_p()
        check(self.lib.fppg_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def set_launch(self, force_block: int = 256, xcd_remap: int = 1, persistent: bool = False):
        """Launch shape (fppg_set_launch; xcd_remap 0 round-robin, 1 one contiguous
        range per XCD, 2 runs of chunks) and schedule (fppg_set_schedule) of the force kernel."""
        check(self.lib.fppg_set_launch(self.handle, int(force_block), int(xcd_remap)), self.handle)
        check(self.lib.fppg_set_schedule(self.handle, int(bool(persistent))), self.handle)

    def close(self):
        if self.handle:
            self.lib.fppg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Geometry:
    """fppg_geom_create / fppg_geom_destroy for a batch of geometries."""

    def __init__(self, ctx: Context, geoms):
        arr, keep = geom_descs(geoms)
        h = ctypes.c_void_p()
        check(ctx.lib.fppg_geom_create(ctx.handle, arr, len(geoms), ctypes.byref(h)), ctx.handle)
        self.ctx = ctx
        self.handle = h
        vals = [ctypes.c_int64() for _ in range(5)]
        check(ctx.lib.fppg_geom_info(h, *[ctypes.byref(v) for v in vals]))
        self.ncell, self.n_tri, self.n_seg, self.search_cells, self.search_entries = (v.value for v in vals)
        self.n_geom = len(geoms)

    def workspace_size(self, n: int) -> int:
        b = ctypes.c_size_t()
        check(self.ctx.lib.fppg_workspace_size(self.handle, int(n), ctypes.byref(b)))
        return int(b.value)

    def close(self):
        if self.handle:
            self.ctx.lib.fppg_geom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Relaxer:
    """Device state and the per-iteration calls for one batch (see module doc)."""

    def __init__(self, wl, device: int = 0, ctx: Context | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("Relaxer needs a GPU (HIP device); none is available")
        self.dev = torch.device("cuda", device)
        self.ctx = ctx or Context(device)
        self.geom = Geometry(self.ctx, wl.geoms)
        self.n = int(wl.n)
        self.na = self.n   # active particles (a tier's reached prefix, see tier())
        self.n_feat = int(len(wl.feat_seg))
        self.move_mask = int(wl.move_mask)
        self.h_min = min(float(g.h) for g in wl.geoms)
        self.n_vert = sum(len(g.mesh.vert) for g in wl.geoms)
        self.vert = np.concatenate([np.asarray(g.mesh.vert, np.float64) for g in wl.geoms], 0)
        pos = np.zeros((self.n, 4), np.float32)
        pos[:, :3] = wl.pos
        pos[:, 3] = _pack_w(wl.tag, wl.gid, getattr(wl, "level", None))
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev, dt)
        self.pos = t(pos, torch.float32)
        self.id = t(np.arange(self.n, dtype=np.int32), torch.int32)
        self.owner = t(wl.owner.astype(np.int32), torch.int32)
        self.pos_b = torch.empty_like(self.pos)
        self.id_b = torch.empty_like(self.id)
        self.owner_b = torch.empty_like(self.owner)
        self.feat_seg = t(wl.feat_seg.astype(np.int32), torch.int32) if self.n_feat else \
            torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.feat_u = t(wl.feat_u.astype(np.float64), torch.float64) if self.n_feat else \
            torch.zeros(1, dtype=torch.float64, device=self.dev)
        self.cell_start = torch.zeros(self.geom.ncell + 2, dtype=torch.int32, device=self.dev)
        self.accel = torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev)
        self.disp = torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev)
        self.amax = torch.zeros(self.geom.n_geom, dtype=torch.float32, device=self.dev)
        self.counters = torch.zeros(L.NCOUNTERS, dtype=torch.int64, device=self.dev)
        self.ws_bytes = self.geom.workspace_size(self.n)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        # receiver list (opt-in): only the moving particles' lanes are launched
        self.use_list = False
        self._tag_counts = np.bincount(np.asarray(wl.tag, np.int64), minlength=8)
        self.mlist = torch.zeros(max(self.n, 1), dtype=torch.int32, device=self.dev)
        self.mcount = torch.zeros(1, dtype=torch.int32, device=self.dev)

    def n_moving(self) -> int:
        """Particles that move under the current move_mask (classes 1..3)."""
        return int(sum(self._tag_counts[t] for t in (1, 2, 3) if (self.move_mask >> t) & 1))

    # ---- the four entry points -------------------------------------------------------------
    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    def build_cells(self):
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_build_cells(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.id), ptr(self.owner),
                                   ptr(self.pos_b), ptr(self.id_b), ptr(self.owner_b), ptr(self.cell_start),
                                   self.ws_ptr, self.ws_bytes, self.stream), c)
        self.pos, self.pos_b = self.pos_b, self.pos
        self.id, self.id_b = self.id_b, self.id
        self.owner, self.owner_b = self.owner_b, self.owner
        if self.use_list:
            self.moving_list()

    def tier(self, move_mask: int, compact: bool = True) -> int:
        """Switch to the tier in which the classes of move_mask move. With
        compact, the particles that the tier does not reach (rank above its
        highest moving class: neither receivers nor sources) are partitioned
        behind the others and left out of every call until the next tier;
        returns the number of active particles."""
        lib, c = self.ctx.lib, self.ctx.handle
        self.release_graph()   # a captured graph holds the previous tier's mask and count
        self.move_mask = int(move_mask)
        mm = self.move_mask if compact else (1 << 3)   # volume bit: every particle active
        na = ctypes.c_int64()
        check(lib.fppg_tier_partition(c, self.geom.handle, self.n, ptr(self.pos), ptr(self.id), ptr(self.owner),
                                      ptr(self.pos_b), ptr(self.id_b), ptr(self.owner_b), mm, ctypes.byref(na),
                                      self.ws_ptr, self.ws_bytes, self.stream), c)
        self.pos, self.pos_b = self.pos_b, self.pos
        self.id, self.id_b = self.id_b, self.id
        self.owner, self.owner_b = self.owner_b, self.owner
        self.na = int(na.value)
        return self.na

    def moving_list(self):
        """Sorted indices of the moving particles into self.mlist (count in self.mcount)."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_moving_list(c, self.geom.handle, self.na, ptr(self.pos), self.move_mask, ptr(self.mlist),
                                   ptr(self.mcount), self.ws_ptr, self.ws_bytes, self.stream), c)

    def volume_layers(self, width: float) -> int:
        """Three-layer volume relaxation: volume particles at distance >= width from the surface become fixed
        (the core); returns how many. The others remain volume particles (the layer a volume tier relaxes)."""
        lib, c = self.ctx.lib, self.ctx.handle
        cnt = torch.zeros(1, dtype=torch.int32, device=self.dev)
        check(lib.fppg_volume_layers(c, self.geom.handle, self.na, ptr(self.pos), float(width), ptr(cnt),
                                     self.stream), c)
        k = int(cnt.cpu()[0])
        self._tag_counts[3] -= k
        self._tag_counts[4] += k
        return k

    def _list_args(self):
        return (ptr(self.mlist), self.n_moving()) if self.use_list else (None, 0)

    def relax_step(self, count_pairs: bool = False, keep_accel: bool = True, forces_only: bool = False):
        """Forces, amax and (unless forces_only) the displacement of every receiver."""
        lib, c = self.ctx.lib, self.ctx.handle
        flags = (L.F_COUNT_PAIRS if count_pairs else 0) | (L.F_FORCES_ONLY if forces_only else 0)
        if forces_only and not keep_accel:
            raise ValueError("forces_only needs keep_accel")
        check(lib.fppg_relax_step(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.owner), ptr(self.cell_start),
                                  ptr(self.feat_seg), self.n_feat, self.move_mask, flags,
                                  ptr(self.accel) if keep_accel else None, ptr(self.amax), ptr(self.disp),
                                  *self._list_args(), self.ws_ptr, self.ws_bytes, self.stream), c)

    def project(self):
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_project(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.owner), ptr(self.disp),
                               ptr(self.feat_seg), ptr(self.feat_u), self.n_feat, self.move_mask,
                               ptr(self.counters), *self._list_args(), self.ws_ptr, self.ws_bytes, self.stream), c)

    def project_record(self, accepted: torch.Tensor):
        """project() that also writes accepted [N] uint8 (1 = the particle's move was applied)."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_project_record(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.owner), ptr(self.disp),
                                      ptr(self.feat_seg), ptr(self.feat_u), self.n_feat, self.move_mask,
                                      ptr(self.counters), ptr(accepted), self.ws_ptr, self.ws_bytes, self.stream), c)

    def hvp(self, v: torch.Tensor, transpose: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
        """J v (or J^T v) for v [N, 4] float32 in the current (sorted) order."""
        lib, c = self.ctx.lib, self.ctx.handle
        out = torch.empty_like(v) if out is None else out
        check(lib.fppg_relax_hvp(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.cell_start),
                                 self.move_mask, int(bool(transpose)), ptr(v), ptr(out), self.stream), c)
        return out

    # ---- Newton-Krylov building blocks ---------------------------------------------------------
    def _scalar(self):
        if not hasattr(self, "_d_scalar"):
            self._d_scalar = torch.zeros(2, dtype=torch.float64, device=self.dev)
        return self._d_scalar

    def energy(self) -> float:
        """Pair energy E of the moving particles at the current state (cells must be current)."""
        lib, c = self.ctx.lib, self.ctx.handle
        out = self._scalar()
        check(lib.fppg_relax_energy(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.cell_start),
                                    self.move_mask, ptr(out), self.ws_ptr, self.ws_bytes, self.stream), c)
        return float(out[0].item())

    def dot(self, a: torch.Tensor, b: torch.Tensor) -> float:
        lib, c = self.ctx.lib, self.ctx.handle
        out = self._scalar()
        check(lib.fppg_vec_dot(c, self.na, ptr(a), ptr(b), ptr(out), self.ws_ptr, self.ws_bytes, self.stream), c)
        return float(out[0].item())

    def axpby(self, alpha: float, x: torch.Tensor, beta: float, y: torch.Tensor):
        """y <- alpha x + beta y (in place)."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_vec_axpby(c, self.na, float(alpha), ptr(x), float(beta), ptr(y), self.stream), c)

    def maxnorm(self, a: torch.Tensor) -> float:
        lib, c = self.ctx.lib, self.ctx.handle
        out = self._scalar()
        check(lib.fppg_vec_maxnorm(c, self.na, ptr(a), ptr(out), self.stream), c)
        return float(out.view(torch.float32)[0].item())

    def clamp(self, v: torch.Tensor, cap: float):
        """Cap every row of v at length `cap` (in place)."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_vec_clamp(c, self.na, ptr(v), float(cap), self.stream), c)

    def hvp_projected(self, v: torch.Tensor, scale: float, out: torch.Tensor) -> torch.Tensor:
        """out = scale P (J v) in one sweep (cells must be current)."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_relax_hvp_projected(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.cell_start),
                                           ptr(self.owner), ptr(self.feat_seg), self.n_feat, self.move_mask,
                                           ptr(v), float(scale), ptr(out), self.stream), c)
        return out

    def combine3(self, a, x, b, y, c3, z, out, phi=0.0, acc=None):
        """out = a x + b y + c3 z; acc += phi out if acc is given."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_vec_combine3(c, self.na, float(a), ptr(x), float(b), ptr(y), float(c3), ptr(z), ptr(out),
                                    float(phi), ptr(acc), self.stream), c)

    def tangent(self, v: torch.Tensor):
        """v <- P v (tangent spaces of the constrained particles; 0 where nothing moves)."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_tangent_project(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.owner),
                                       ptr(self.feat_seg), self.n_feat, self.move_mask, ptr(v), self.stream), c)

    def displace(self, v: torch.Tensor, alpha: float):
        """self.disp <- alpha P v in the displacement format that project() applies."""
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_displace(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.owner), ptr(self.feat_seg),
                                self.n_feat, self.move_mask, ptr(v), float(alpha), ptr(self.disp), self.stream), c)

    def snapshot(self):
        """Device copies of the mutable state (positions, ids, owners, feature table, cells)."""
        return (self.pos.clone(), self.id.clone(), self.owner.clone(), self.feat_seg.clone(),
                self.feat_u.clone(), self.cell_start.clone())

    def restore(self, snap):
        for dst, src in zip((self.pos, self.id, self.owner, self.feat_seg, self.feat_u, self.cell_start), snap):
            dst.copy_(src)
        if self.use_list:
            # the receiver list indexes the sorted order: rebuild it for the restored order
            self.moving_list()

    def neighbors(self, cap: int = 160):
        lib, c = self.ctx.lib, self.ctx.handle
        count = torch.zeros(self.n, dtype=torch.int32, device=self.dev)
        lst = torch.full((self.n, cap), -1, dtype=torch.int32, device=self.dev)
        check(lib.fppg_debug_neighbors(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.cell_start),
                                       ptr(count), ptr(lst), cap, self.stream), c)
        return count, lst

    def profile(self, enable: bool = True, phases=None):
        """Time the phases (names of L.PHASES, default all) of the per-iteration calls with HIP events on the
        launch stream; enable=False stops."""
        mask = 0
        if enable:
            mask = (1 << L.NPHASES) - 1 if phases is None else sum(1 << L.PHASES.index(p) for p in phases)
        check(self.ctx.lib.fppg_profile(self.ctx.handle, mask), self.ctx.handle)

    def profile_read(self) -> dict:
        """{phase: (total ms, launches)} since profiling was enabled."""
        ms = (ctypes.c_double * L.NPHASES)()
        cnt = (ctypes.c_int64 * L.NPHASES)()
        check(self.ctx.lib.fppg_profile_read(self.ctx.handle, ms, cnt), self.ctx.handle)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.PHASES)}

    def read_status(self) -> int:
        f = ctypes.c_uint32()
        check(self.ctx.lib.fppg_read_status(self.ctx.handle, self.stream, ctypes.byref(f)), self.ctx.handle)
        return int(f.value)

    # ---- loop -------------------------------------------------------------------------------
    def step(self, count_pairs: bool = False, keep_accel: bool = True):
        """One iteration of Algorithm 1."""
        self.build_cells()
        self.relax_step(count_pairs=count_pairs, keep_accel=keep_accel)
        self.project()

    def run(self, iters: int):
        for _ in range(iters):
            self.step(keep_accel=False)

    # ---- graph capture -----------------------------------------------------------------------
    def capture(self, iters: int = 2):
        """Capture `iters` (even) iterations into a HIP graph on a side stream."""
        self.release_graph()
        self.graph_stream = torch.cuda.Stream(device=self.dev)
        self.graph_stream.wait_stream(torch.cuda.current_stream(self.dev))
        lib, c = self.ctx.lib, self.ctx.handle
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(self.graph_stream.cuda_stream)
        check(lib.fppg_graph_create(c, self.geom.handle, self.na, ptr(self.pos), ptr(self.id), ptr(self.owner),
                                    ptr(self.pos_b), ptr(self.id_b), ptr(self.owner_b), ptr(self.cell_start),
                                    ptr(self.feat_seg), ptr(self.feat_u), self.n_feat, self.move_mask,
                                    ptr(self.amax), ptr(self.disp), ptr(self.counters), self.ws_ptr,
                                    self.ws_bytes, int(iters), st, ctypes.byref(h)), c)
        self.graph = h
        self.graph_iters = int(iters)
        self._graph_a = self.pos.data_ptr()

    def replay(self, repeats: int = 1):
        """Run repeats * graph_iters iterations from the captured graph (state ends in the same buffers)."""
        if not getattr(self, "graph", None):
            raise RuntimeError("no captured graph (capture() first; tier() releases it)")
        cur = torch.cuda.current_stream(self.dev)
        if self.pos.data_ptr() != self._graph_a:
            # an odd number of eager rebuilds since the capture left the state in
            # buffer set B: move it back to set A, which the graph reads
            self.pos_b.copy_(self.pos)
            self.id_b.copy_(self.id)
            self.owner_b.copy_(self.owner)
            self.pos, self.pos_b = self.pos_b, self.pos
            self.id, self.id_b = self.id_b, self.id
            self.owner, self.owner_b = self.owner_b, self.owner
        self.graph_stream.wait_stream(cur)
        lib, c = self.ctx.lib, self.ctx.handle
        check(lib.fppg_graph_launch(c, self.graph, int(repeats), ctypes.c_void_p(self.graph_stream.cuda_stream)), c)
        cur.wait_stream(self.graph_stream)

    def release_graph(self):
        if getattr(self, "graph", None):
            self.ctx.lib.fppg_graph_destroy(self.graph)
            self.graph = None

    # ---- host views (by particle id) ---------------------------------------------------------
    def host_state(self):
        """(pos32 [N,3], owner [N], feat_seg, feat_u) ordered by particle id."""
        torch.cuda.synchronize(self.dev)
        ids = self.id.cpu().numpy()
        pos = self.pos.cpu().numpy()
        own = self.owner.cpu().numpy()
        p = np.empty((self.n, 3), np.float32)
        o = np.empty(self.n, np.int32)
        p[ids] = pos[:, :3]
        o[ids] = own
        fs = self.feat_seg.cpu().numpy()[: self.n_feat].copy()
        fu = self.feat_u.cpu().numpy()[: self.n_feat].copy()
        return p, o, fs, fu

    def by_id(self, t: torch.Tensor) -> np.ndarray:
        """Rows of a per-particle tensor in the current order, re-ordered by id."""
        torch.cuda.synchronize(self.dev)
        ids = self.id.cpu().numpy()
        a = t.detach().cpu().numpy()
        out = np.empty_like(a)
        out[ids] = a
        return out
