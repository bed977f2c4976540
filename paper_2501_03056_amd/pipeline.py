"""A mesh to relaxation-ready particles on the GPU: fppg_features (feature
lines, singular points, feature-line particles) and fppg_generate (volume
particles at internal cell centres, surface particles mapped onto facets),
assembled into the particle state and geometry description a Relaxer takes.

The assembly only lays out the kernels' outputs (class tags, owner indices,
the feature table, the particle-grid constants); the particles themselves all
come from the two kernels.
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np
import torch

from . import front

SINGULAR, FEATURE, SURFACE, VOLUME = 0, 1, 2, 3
ALL_MOVING = (1 << FEATURE) | (1 << SURFACE) | (1 << VOLUME)


def _f32(x) -> float:
    return float(np.float32(x))


def particle_grid(lo, hi, h, k=2, pad=None):
    """Particle-grid constants covering [lo, hi] with a margin of `pad` (one
    support radius by default): cell edge (2h/k)(1 + 2^-8) in binary32."""
    rc = _f32(2.0 * h)
    pad = rc if pad is None else pad
    cell = _f32((rc / k) * (1.0 + 2.0 ** -8))
    inv = _f32(1.0 / cell)
    origin = (np.asarray(lo, np.float64) - pad).astype(np.float32)
    ext = np.asarray(hi, np.float64) + pad - origin.astype(np.float64)
    dims = np.ceil(ext * inv).astype(np.int64) + 1
    return origin, inv, dims


class _Workload(SimpleNamespace):
    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def n_moving(self) -> int:
        return int(np.sum((self.move_mask >> self.tag) & 1))

    def counts(self) -> dict:
        names = ["singular", "feature", "surface", "volume", "fixed"]
        return {nm: int(np.sum(self.tag == t)) for t, nm in enumerate(names)}


def from_mesh(vert, tri, dx: float, cos_threshold: float = math.cos(math.radians(30.0)), k: int = 2,
              h_over_dx: float = 1.3, device: int = 0, ctx=None, name: str = "mesh"):
    """Particles of a closed mesh at spacing dx, ready for Relaxer(...): the
    generation grid is the mesh's bounding box widened by 2 dx."""
    vert = np.ascontiguousarray(vert, np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
    ctx = ctx or front.Context(device)
    f = front.features(vert, tri, cos_threshold, dx, ctx=ctx)
    lo, hi = vert.min(0) - 2 * dx, vert.max(0) + 2 * dx
    dims = tuple(int(v) for v in np.ceil((hi - lo) / dx))
    cls, gpos, gown = front.generate(vert, tri, dx, lo, dims, ctx=ctx)
    # feature lines as segments (vertex k to k + 1, a loop closed by its first vertex)
    lb = f["line_begin"].cpu().numpy()
    lv = f["line_vert"].cpu().numpy()
    closed = f["line_closed"].cpu().numpy().astype(np.uint8)
    seg_begin, seg_p, seg_vert = [0], [], []
    for l in range(len(lb) - 1):
        vs = lv[lb[l]:lb[l + 1]].tolist()
        if closed[l]:
            vs = vs + vs[:1]
        for a, b in zip(vs[:-1], vs[1:]):
            seg_p.append((vert[a], vert[b]))
            seg_vert.append((a, b))
        seg_begin.append(len(seg_p))
    lines = SimpleNamespace(line_seg_begin=np.array(seg_begin, np.int32),
                            seg_p=np.array(seg_p, np.float64).reshape(-1, 2, 3), line_closed=closed,
                            seg_vert=np.array(seg_vert, np.int32).reshape(-1, 2))
    lines.n_line = len(closed)
    lines.n_seg = len(seg_p)
    mesh = SimpleNamespace(vert=vert, tri=tri, lines=lines)
    # particles: singular, feature, surface and volume
    sing = f["singular"].cpu().numpy().astype(np.int64)
    fpos = f["pos"].cpu().numpy()[:, :3]
    fline = f["line_of"].cpu().numpy().astype(np.int64)
    fseg = f["seg"].cpu().numpy().astype(np.int64)
    fu = f["u"].cpu().numpy()
    gp = gpos.cpu().numpy()
    gtag = gp[:, 3].copy().view(np.int32) & 7
    gown = gown.cpu().numpy()
    n_f = len(fpos)
    pos = np.concatenate([vert[sing].astype(np.float32), fpos, gp[:, :3]], 0).astype(np.float32)
    tag = np.concatenate([np.full(len(sing), SINGULAR), np.full(n_f, FEATURE), gtag]).astype(np.int32)
    owner = np.concatenate([sing, np.arange(n_f), gown]).astype(np.int32)
    feat_seg = (np.array(seg_begin, np.int64)[fline] + fseg).astype(np.int32)
    h = _f32(h_over_dx * dx)
    origin, inv, gdims = particle_grid(vert.min(0), vert.max(0), h, k)
    geo = SimpleNamespace(mesh=mesh, dx=dx, h=h, k=k, proj_radius=_f32(dx), origin=origin, inv_cell=inv,
                          dims=gdims, part_begin=0, part_end=len(pos), tri_begin=0, seg_begin=0,
                          line_begin=0, feat_begin=0, vert_begin=0, slab=0)
    wl = _Workload(name=name, geoms=[geo], pos=pos, tag=tag, owner=owner, gid=np.zeros(len(pos), np.int32),
                   feat_seg=feat_seg, feat_u=fu.astype(np.float64), move_mask=ALL_MOVING, seed=0,
                   meta={"generation_cells": cls.cpu().numpy()})
    return wl
