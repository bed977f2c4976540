"""Seeded synthetic workloads: meshes plus an initial (unrelaxed) particle cloud.

The paper seeds particles at the centres of internal and surface grid cells,
maps surface seeds onto facets and places feature-line particles at a spacing
that divides each line evenly (section 3.2). Its models are not available, so
this module builds stand-ins with the same structure: a jittered lattice of
volume particles clipped to the inside, surface particles lying exactly on
facets (with the owning facet recorded), feature particles on the sharp-edge
polylines (with their segment and arc-length coordinate), and fixed singular
particles at corners. All randomness comes from numpy's PCG64 with a stated
seed.

Particle tags (the particle classes of section 2.2 / 3.3):
  0 singular point (never moves)   1 feature-line particle
  2 surface particle                3 volume particle
  4 fixed volume particle (innermost layer of the narrow band, never moves)

Owner: facet index (global over the batch) for surface particles, feature slot
for feature particles, -1 otherwise.

This module is an input generator shared by the oracle and the GPU path; it
performs none of the relaxation method's arithmetic.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass, field

import numpy as np

from . import csg as C
from . import meshes as M

SINGULAR, FEATURE, SURFACE, VOLUME, FIXED = 0, 1, 2, 3, 4
ALL_MOVING = (1 << FEATURE) | (1 << SURFACE) | (1 << VOLUME)


def f32(x) -> float:
    """Round a Python float to the nearest binary32 value (returned as float)."""
    return float(np.float32(x))


@dataclass
class Geometry:
    """One geometry of a batch: its mesh and the particle-grid description.

    The particle grid is a uniform Cartesian grid of cell edge (2h/k)(1+2^-8)
    starting at `origin` with `dims` cells per axis (the relaxation keys its
    own cells from it).
    """
    mesh: M.Mesh
    dx: float
    h: float              # binary32 value
    k: int
    proj_radius: float    # binary32 value
    origin: np.ndarray    # float32 [3]
    inv_cell: float       # binary32 value
    dims: np.ndarray      # int64 [3]
    part_begin: int = 0
    part_end: int = 0
    tri_begin: int = 0
    seg_begin: int = 0
    line_begin: int = 0
    feat_begin: int = 0
    vert_begin: int = 0   # global id of the mesh's first vertex (singular-particle owners)
    slab: int = 0         # rows of cells along y per slab of the cell key (0: one slab)
    csg: object = None    # csg.CSG: the mesh is the facets of convex parts combined by a Boolean operation
    max_level: int = 0    # multi-resolution: particle levels 0..max_level, h_i = h 2^-level


def particle_grid(lo, hi, h, k=2, pad=None):
    """Grid parameters covering [lo, hi] plus a margin of one support radius."""
    rc = f32(2.0 * h)
    pad = rc if pad is None else pad
    cell = f32((rc / k) * (1.0 + 2.0 ** -8))
    inv = f32(1.0 / cell)
    origin = (np.asarray(lo, np.float64) - pad).astype(np.float32)
    ext = np.asarray(hi, np.float64) + pad - origin.astype(np.float64)
    dims = np.ceil(ext * inv).astype(np.int64) + 1
    return origin, inv, dims


@dataclass
class Workload:
    name: str
    geoms: list
    pos: np.ndarray        # float32 [N, 3]
    tag: np.ndarray        # int32 [N]
    owner: np.ndarray      # int32 [N]
    gid: np.ndarray        # int32 [N] geometry index
    feat_seg: np.ndarray   # int32 [n_feat] global segment index
    feat_u: np.ndarray     # float64 [n_feat] arc length inside the segment
    move_mask: int = ALL_MOVING
    seed: int = 0
    meta: dict = field(default_factory=dict)
    level: np.ndarray = None   # int32 [N] resolution level (multi-resolution geometries), None: all 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def ids(self) -> np.ndarray:
        return np.arange(self.n, dtype=np.int32)

    def n_moving(self) -> int:
        return int(np.sum((self.move_mask >> self.tag) & 1))

    def counts(self) -> dict:
        names = ["singular", "feature", "surface", "volume", "fixed"]
        return {nm: int(np.sum(self.tag == t)) for t, nm in enumerate(names)}


class _Builder:
    """Accumulates particles of one geometry."""

    def __init__(self):
        self.pos, self.tag, self.owner = [], [], []
        self.feat_seg, self.feat_u = [], []

    def add(self, pos, tag, owner=None):
        pos = np.asarray(pos, np.float64).reshape(-1, 3)
        self.pos.append(pos)
        self.tag.append(np.full(len(pos), tag, np.int32))
        self.owner.append(np.full(len(pos), -1, np.int32) if owner is None
                          else np.asarray(owner, np.int32))

    def add_feature(self, pos, seg, u):
        base = sum(len(s) for s in self.feat_seg)
        self.feat_seg.append(np.asarray(seg, np.int32))
        self.feat_u.append(np.asarray(u, np.float64))
        self.add(pos, FEATURE, base + np.arange(len(seg)))


def _seg_table(lines: M.FeatureLines):
    p0, p1 = lines.seg_p[:, 0], lines.seg_p[:, 1]
    ln = np.linalg.norm(p1 - p0, axis=1)
    return p0, p1, ln


def _feature_particles(b: _Builder, mesh: M.Mesh, dx: float, rng, jitter: float):
    """Particles along every feature line at spacing L/ceil(L/dx) (section 3.2.2).

    Open lines exclude their end points (those are singular points); loops
    place ceil(L/dx) particles. Each gets a uniform jitter along the line.
    """
    lines = mesh.lines
    p0, p1, ln = _seg_table(lines)
    for l in range(lines.n_line):
        s0, s1 = lines.line_seg_begin[l], lines.line_seg_begin[l + 1]
        seg_len = ln[s0:s1]
        cum = np.concatenate([[0.0], np.cumsum(seg_len)])
        L = cum[-1]
        m = max(int(np.ceil(L / dx)), 1)
        sp = L / m
        if lines.line_closed[l]:
            s = (np.arange(m) + 0.5) * sp
        else:
            s = np.arange(1, m) * sp
        if len(s) == 0:
            continue
        s = s + rng.uniform(-jitter, jitter, len(s)) * sp
        if lines.line_closed[l]:
            s = np.mod(s, L)
        k = np.clip(np.searchsorted(cum, s, side="right") - 1, 0, len(seg_len) - 1)
        u = s - cum[k]
        u = np.clip(u, 0.0, seg_len[k])
        seg = s0 + k
        t = (p1[seg] - p0[seg]) / ln[seg][:, None]
        pos = p0[seg] + u[:, None] * t
        b.add_feature(pos, seg, u)


def _finish(name, parts, move_mask, seed, meta=None) -> Workload:
    """Concatenate per-geometry builders into one workload with global offsets."""
    geoms, pos, tag, owner, gid, fseg, fu = [], [], [], [], [], [], []
    n = tri_off = seg_off = line_off = feat_off = vert_off = 0
    for g, (geom, b) in enumerate(parts):
        p = np.concatenate(b.pos, 0) if b.pos else np.zeros((0, 3))
        t = np.concatenate(b.tag) if b.tag else np.zeros(0, np.int32)
        o = np.concatenate(b.owner) if b.owner else np.zeros(0, np.int32)
        o = o.copy()
        o[t == SURFACE] += tri_off
        o[t == FEATURE] += feat_off
        o[t == SINGULAR] += vert_off
        geom.part_begin, geom.part_end = n, n + len(p)
        geom.tri_begin, geom.seg_begin, geom.line_begin = tri_off, seg_off, line_off
        geom.feat_begin, geom.vert_begin = feat_off, vert_off
        geoms.append(geom)
        pos.append(p.astype(np.float32))
        tag.append(t)
        owner.append(o)
        gid.append(np.full(len(p), g, np.int32))
        if b.feat_seg:
            fseg.append(np.concatenate(b.feat_seg) + seg_off)
            fu.append(np.concatenate(b.feat_u))
            feat_off += len(fseg[-1])
        n += len(p)
        tri_off += geom.mesh.n_tri
        seg_off += geom.mesh.lines.n_seg
        line_off += geom.mesh.lines.n_line
        vert_off += len(geom.mesh.vert)
    return Workload(
        name=name, geoms=geoms, pos=np.concatenate(pos, 0), tag=np.concatenate(tag),
        owner=np.concatenate(owner), gid=np.concatenate(gid),
        feat_seg=(np.concatenate(fseg) if fseg else np.zeros(0, np.int32)).astype(np.int32),
        feat_u=np.concatenate(fu) if fu else np.zeros(0, np.float64),
        move_mask=move_mask, seed=seed, meta=meta or {})


def _make_geom(mesh, dx, k=2, proj_radius=None):
    h = f32(1.3 * dx)
    lo, hi = mesh.bbox()
    origin, inv, dims = particle_grid(lo, hi, h, k)
    # R = dx: the facet search cells are the background grid of the
    # generation (one particle spacing), whose 27 cells the reprojection of
    # section 3.3.3 searches
    R = f32(dx) if proj_radius is None else f32(proj_radius)
    return Geometry(mesh=mesh, dx=dx, h=h, k=k, proj_radius=R, origin=origin,
                    inv_cell=inv, dims=dims)


# ---------------------------------------------------------------------------
# Unit cube
# ---------------------------------------------------------------------------

def _tri_owner_on_plane(mesh: M.Mesh, cand: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Index (into cand) of the candidate facet containing each point (points on the facet planes)."""
    A = mesh.vert[mesh.tri[cand, 0]]
    B = mesh.vert[mesh.tri[cand, 1]]
    C = mesh.vert[mesh.tri[cand, 2]]
    out = np.full(len(pts), -1, np.int64)
    for c in range(len(cand)):
        n = np.cross(B[c] - A[c], C[c] - A[c])
        s0 = np.cross(B[c] - A[c], pts - A[c]) @ n
        s1 = np.cross(C[c] - B[c], pts - B[c]) @ n
        s2 = np.cross(A[c] - C[c], pts - C[c]) @ n
        inside = (s0 >= 0) & (s1 >= 0) & (s2 >= 0) & (out < 0)
        out[inside] = c
    return out


def cube_workload(n=24, jitter=0.3, seed=1, k=2, with_volume=True, with_surface=True,
                  with_features=True, move_mask=ALL_MOVING, name=None) -> Workload:
    """Unit cube [0,1]^3, dx = 1/n: a jittered (i+1/2)dx lattice of volume
    particles, (a+1/2)dx x (b+1/2)dx surface particles per face with tangential
    jitter, features at m*dx along the 12 edges, fixed particles at the 8 corners."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mesh = M.cube()
    dx = 1.0 / n
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    c = (np.arange(n) + 0.5) * dx
    if with_volume:
        g = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
        g = g + rng.uniform(-jitter, jitter, g.shape) * dx
        b.add(g, VOLUME)
    if with_surface:
        nrm = np.cross(mesh.vert[mesh.tri[:, 1]] - mesh.vert[mesh.tri[:, 0]],
                       mesh.vert[mesh.tri[:, 2]] - mesh.vert[mesh.tri[:, 0]])
        for axis in range(3):
            u, v = [a for a in range(3) if a != axis]
            for side in (0.0, 1.0):
                uu, vv = np.meshgrid(c, c, indexing="ij")
                pts = np.zeros((n * n, 3))
                pts[:, u] = uu.ravel() + rng.uniform(-jitter, jitter, n * n) * dx
                pts[:, v] = vv.ravel() + rng.uniform(-jitter, jitter, n * n) * dx
                pts[:, axis] = side
                want = np.zeros(3)
                want[axis] = 1.0 if side == 1.0 else -1.0
                cand = np.nonzero(np.isclose(nrm @ want, np.linalg.norm(nrm, axis=1)))[0]
                own = _tri_owner_on_plane(mesh, cand, pts)
                assert (own >= 0).all()
                b.add(pts, SURFACE, cand[own])
    if with_features:
        _feature_particles(b, mesh, dx, rng, jitter)
        b.add(mesh.singular, SINGULAR, mesh.singular_vert)
    return _finish(name or f"cube_n{n}", [(geom, b)], move_mask, seed,
                   {"dx": dx, "jitter": jitter})


def dyadic_lattice_workload(m=16, dx=2.0 ** -5, k=2) -> Workload:
    """Exact lattice of m^3 volume particles at (i+1/2)dx, no jitter, no mesh
    constraints exercised: every coordinate is a binary32 value."""
    mesh = M.cube((0.0, 0.0, 0.0), (m * dx, m * dx, m * dx))
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    c = (np.arange(m) + 0.5) * dx
    g = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    b.add(g, VOLUME)
    return _finish(f"dyadic_m{m}", [(geom, b)], 1 << VOLUME, 0, {"dx": dx})


# ---------------------------------------------------------------------------
# Sphere
# ---------------------------------------------------------------------------

def _facet_planes(mesh):
    A = mesh.vert[mesh.tri[:, 0]]
    B = mesh.vert[mesh.tri[:, 1]]
    C = mesh.vert[mesh.tri[:, 2]]
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1)[:, None]
    return A, B, C, n


def _radial_map_sphere(mesh: M.Mesh, dirs: np.ndarray):
    """Map unit directions from the origin onto the facet the ray hits."""
    from scipy.spatial import cKDTree
    A, B, C, n = _facet_planes(mesh)
    cen = (A + B + C) / 3
    cen /= np.linalg.norm(cen, axis=1)[:, None]
    tree = cKDTree(cen)
    _, cand = tree.query(dirs, k=8)
    owner = np.full(len(dirs), -1, np.int64)
    for c in range(cand.shape[1]):
        t = cand[:, c]
        s0 = np.einsum("ij,ij->i", np.cross(A[t], B[t]), dirs)
        s1 = np.einsum("ij,ij->i", np.cross(B[t], C[t]), dirs)
        s2 = np.einsum("ij,ij->i", np.cross(C[t], A[t]), dirs)
        ok = (s0 >= 0) & (s1 >= 0) & (s2 >= 0) & (owner < 0)
        owner[ok] = t[ok]
    assert (owner >= 0).all(), "radial map: direction outside all candidate facets"
    s = np.einsum("ij,ij->i", n[owner], A[owner]) / np.einsum("ij,ij->i", n[owner], dirs)
    return dirs * s[:, None], owner


def fibonacci_sphere(m: int) -> np.ndarray:
    i = np.arange(m) + 0.5
    z = 1.0 - 2.0 * i / m
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def sphere_workload(level=5, dx=0.01, jitter=0.3, seed=2, k=2, with_volume=True,
                    with_surface=True, move_mask=ALL_MOVING, name=None) -> Workload:
    """Icosphere of radius 1. Volume: jittered (i+1/2)dx lattice on [-1,1]^3 kept
    where the distance to the mesh is at least dx/2 inside (tested against the
    inscribed radius of the mesh). Surface: round(4 pi / dx^2) Fibonacci
    directions with tangential jitter, mapped radially onto the facet they hit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mesh = M.icosphere(level)
    geom = _make_geom(mesh, dx, k)
    A, B, C, n = _facet_planes(mesh)
    r_in = float(np.min(np.einsum("ij,ij->i", n, A)))
    b = _Builder()
    if with_volume:
        m = int(round(2.0 / dx))
        c = -1.0 + (np.arange(m) + 0.5) * dx
        keep = []
        for ix in range(m):  # slab by slab to bound memory
            yy, zz = np.meshgrid(c, c, indexing="ij")
            g = np.stack([np.full(yy.size, c[ix]), yy.ravel(), zz.ravel()], 1)
            g = g + rng.uniform(-jitter, jitter, g.shape) * dx
            keep.append(g[np.linalg.norm(g, axis=1) <= r_in - 0.5 * dx])
        b.add(np.concatenate(keep, 0), VOLUME)
    if with_surface:
        ms = int(round(4.0 * np.pi / dx ** 2))
        d = fibonacci_sphere(ms)
        d = d + rng.uniform(-jitter, jitter, d.shape) * dx
        d /= np.linalg.norm(d, axis=1)[:, None]
        p, own = _radial_map_sphere(mesh, d)
        b.add(p, SURFACE, own)
    return _finish(name or f"sphere_l{level}_dx{dx:g}", [(geom, b)], move_mask, seed,
                   {"dx": dx, "jitter": jitter, "r_in": r_in})


def multires_sphere_workload(level=3, dx=0.08, shell=2.0, jitter=0.3, seed=2, k=2, move_mask=ALL_MOVING,
                             name=None) -> Workload:
    """Icosphere of radius 1 at two resolutions: a fine shell (level 1,
    spacing dx/2) and a coarse core (level 0, spacing dx). Fine volume
    particles: jittered (i+1/2)(dx/2) lattice with radius in [r_in - shell*dx,
    r_in - dx/4]; coarse ones: jittered (i+1/2)dx lattice with radius below
    r_in - shell*dx - dx/2 (r_in the inscribed radius of the mesh); surface
    particles at the fine spacing (Fibonacci directions mapped radially), level
    1. The geometry's h = 1.3 dx is the coarse length (cells sized by it)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mesh = M.icosphere(level)
    geom = _make_geom(mesh, dx, k)
    geom.max_level = 1
    A, B, C, n = _facet_planes(mesh)
    r_in = float(np.min(np.einsum("ij,ij->i", n, A)))
    b = _Builder()
    lv = []
    for sp, lo_r, hi_r, lev in ((dx, -1.0, r_in - shell * dx - 0.5 * dx, 0),
                                (0.5 * dx, r_in - shell * dx, r_in - 0.25 * dx, 1)):
        m = int(round(2.0 / sp))
        c = -1.0 + (np.arange(m) + 0.5) * sp
        keep = []
        for ix in range(m):
            yy, zz = np.meshgrid(c, c, indexing="ij")
            g = np.stack([np.full(yy.size, c[ix]), yy.ravel(), zz.ravel()], 1)
            g = g + rng.uniform(-jitter, jitter, g.shape) * sp
            r = np.linalg.norm(g, axis=1)
            keep.append(g[(r <= hi_r) & (r >= lo_r)])
        pts = np.concatenate(keep, 0)
        b.add(pts, VOLUME)
        lv.append(np.full(len(pts), lev, np.int32))
    fine = 0.5 * dx
    ms = int(round(4.0 * np.pi / fine ** 2))
    d = fibonacci_sphere(ms)
    d = d + rng.uniform(-jitter, jitter, d.shape) * fine
    d /= np.linalg.norm(d, axis=1)[:, None]
    p, own = _radial_map_sphere(mesh, d)
    b.add(p, SURFACE, own)
    lv.append(np.full(len(p), 1, np.int32))
    wl = _finish(name or f"mr_sphere_l{level}_dx{dx:g}", [(geom, b)], move_mask, seed,
                 {"dx": dx, "jitter": jitter, "r_in": r_in, "shell": shell})
    wl.level = np.concatenate(lv)
    return wl


# ---------------------------------------------------------------------------
# Regular tetrahedron
# ---------------------------------------------------------------------------

def _convex_inside(mesh, pts, margin):
    """Points whose distance to every facet plane is at least `margin` inside (convex mesh)."""
    A, B, C, n = _facet_planes(mesh)
    sd = (pts @ n.T) - np.einsum("ij,ij->i", n, A)[None, :]
    return np.all(sd <= -margin, axis=1)


def tetra_workload(dx=0.045, jitter=0.3, seed=5, k=2, move_mask=ALL_MOVING, name=None) -> Workload:
    """Regular tetrahedron of edge 1. Volume: jittered lattice at least dx/2
    inside. Surface: per face a jittered square lattice in the face plane, kept
    at least dx/2 from the face edges. Features on the 6 edges, 4 singular corners."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mesh = M.tetrahedron()
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    lo, hi = mesh.bbox()
    axes = [np.arange(lo[a] + 0.5 * dx, hi[a], dx) for a in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    g = g + rng.uniform(-jitter, jitter, g.shape) * dx
    b.add(g[_convex_inside(mesh, g, 0.5 * dx)], VOLUME)
    A, B, C, n = _facet_planes(mesh)
    for f in range(mesh.n_tri):
        e0 = (B[f] - A[f]) / np.linalg.norm(B[f] - A[f])
        e1 = np.cross(n[f], e0)
        span = np.arange(-0.5, 1.5, dx)
        uu, vv = np.meshgrid(span, span, indexing="ij")
        uv = np.stack([uu.ravel(), vv.ravel()], 1)
        uv = uv + rng.uniform(-jitter, jitter, uv.shape) * dx
        pts = A[f] + uv[:, :1] * e0 + uv[:, 1:] * e1
        # keep points inside the facet at least dx/2 from its edges
        ok = np.ones(len(pts), bool)
        for (P, Q) in ((A[f], B[f]), (B[f], C[f]), (C[f], A[f])):
            ein = np.cross(n[f], Q - P)
            ein /= np.linalg.norm(ein)
            ok &= (pts - P) @ ein >= 0.5 * dx
        b.add(pts[ok], SURFACE, np.full(int(ok.sum()), f))
    _feature_particles(b, mesh, dx, rng, jitter)
    b.add(mesh.singular, SINGULAR, mesh.singular_vert)
    return _finish(name or f"tetra_dx{dx:g}", [(geom, b)], move_mask, seed, {"dx": dx})


def custom_workload(mesh, dx, pos, tag, owner=None, feat_seg=None, feat_u=None,
                    move_mask=ALL_MOVING, k=2, name="custom") -> Workload:
    """A single-geometry workload from explicit particle arrays (for small cases)."""
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    tag = np.asarray(tag, np.int32).reshape(-1)
    owner = np.full(len(pos), -1, np.int32) if owner is None else np.asarray(owner, np.int32)
    b.pos.append(pos)
    b.tag.append(tag)
    b.owner.append(owner)
    if feat_seg is not None and len(feat_seg):
        b.feat_seg.append(np.asarray(feat_seg, np.int32))
        b.feat_u.append(np.asarray(feat_u, np.float64))
    return _finish(name, [(geom, b)], move_mask, 0, {"dx": dx})


# ---------------------------------------------------------------------------
# Convex solids and the batch of independent geometries
# ---------------------------------------------------------------------------

def _surface_particles_planar(b: _Builder, mesh: M.Mesh, dx: float, rng, jitter: float):
    """Jittered square lattice of spacing dx on every plane of a mesh whose
    faces are planar polygons split into coplanar facets; points kept at least
    dx/2 from the polygon boundary, owner = the facet containing the point."""
    A, B, C, n = _facet_planes(mesh)
    d = np.einsum("ij,ij->i", n, A)
    key = np.round(np.concatenate([n, d[:, None]], 1), 9)
    _, group = np.unique(key, axis=0, return_inverse=True)
    group = group.ravel()
    for gidx in range(group.max() + 1):
        fs = np.nonzero(group == gidx)[0]
        nn = n[fs[0]]
        u = B[fs[0]] - A[fs[0]]
        u /= np.linalg.norm(u)
        v = np.cross(nn, u)
        o = A[fs[0]]
        # boundary edges of the polygon: edges used by one facet of the group
        cnt = {}
        for f in fs:
            t = mesh.tri[f]
            for a, c in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                e = (min(a, c), max(a, c))
                cnt[e] = cnt.get(e, 0) + 1
        bnd = np.array([e for e, k in cnt.items() if k == 1])
        P = mesh.vert[bnd[:, 0]] - o
        Q = mesh.vert[bnd[:, 1]] - o
        p2 = np.stack([P @ u, P @ v], 1)
        q2 = np.stack([Q @ u, Q @ v], 1)
        vs = mesh.vert[np.unique(mesh.tri[fs])] - o
        uv = np.stack([vs @ u, vs @ v], 1)
        lo, hi = uv.min(0), uv.max(0)
        ga = np.arange(lo[0] + 0.5 * dx, hi[0], dx)
        gb = np.arange(lo[1] + 0.5 * dx, hi[1], dx)
        if len(ga) == 0 or len(gb) == 0:
            continue
        g2 = np.stack(np.meshgrid(ga, gb, indexing="ij"), -1).reshape(-1, 2)
        g2 = g2 + rng.uniform(-jitter, jitter, g2.shape) * dx
        # distance to every boundary segment (2-D)
        e = q2 - p2
        w = g2[:, None, :] - p2[None]
        tt = np.clip(np.einsum("pek,ek->pe", w, e) / np.einsum("ek,ek->e", e, e), 0.0, 1.0)
        dist = np.linalg.norm(w - tt[..., None] * e[None], axis=2).min(1)
        g2 = g2[dist >= 0.5 * dx]
        pts = o + g2[:, :1] * u + g2[:, 1:] * v
        own = np.full(len(pts), -1)
        for f in fs:
            la, lb, lc = _bary(pts, A[f], B[f], C[f])
            inside = (np.minimum(np.minimum(la, lb), lc) >= 0) & (own < 0)
            own[inside] = f
        keep = own >= 0
        b.add(pts[keep], SURFACE, own[keep])


def _bary(p, A, B, C):
    e0, e1, w = B - A, C - A, p - A
    d00, d01, d11 = e0 @ e0, e0 @ e1, e1 @ e1
    d20, d21 = w @ e0, w @ e1
    den = d00 * d11 - d01 * d01
    lb = (d11 * d20 - d01 * d21) / den
    lc = (d00 * d21 - d01 * d20) / den
    return 1 - lb - lc, lb, lc


def _convex_volume_particles(b: _Builder, mesh: M.Mesh, dx: float, rng, jitter: float):
    lo, hi = mesh.bbox()
    axes = [np.arange(lo[a] + 0.5 * dx, hi[a], dx) for a in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    g = g + rng.uniform(-jitter, jitter, g.shape) * dx
    b.add(g[_convex_inside(mesh, g, 0.5 * dx)], VOLUME)


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def solid_geometry(rng, n_target: float, jitter=0.3, k=2):
    """One random convex solid (box with edges U(0.1,1), or a 64-segment
    cylinder with diameter and height U(0.1,1)), randomly rotated, with dx set
    so that it holds about n_target particles. Returns (Geometry, _Builder, kind)."""
    if rng.uniform() < 0.5:
        e = rng.uniform(0.1, 1.0, 3)
        mesh = M.cube(-e / 2, e / 2)
        vol = float(np.prod(e))
        kind = "box"
    else:
        dia, hgt = rng.uniform(0.1, 1.0, 2)
        mesh = M.cylinder(dia / 2, hgt, 64)
        vol = float(np.pi * (dia / 2) ** 2 * hgt)
        kind = "cylinder"
    mesh = M.transformed(mesh, _random_rotation(rng), np.zeros(3))
    dx = (vol / n_target) ** (1.0 / 3.0)
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    _convex_volume_particles(b, mesh, dx, rng, jitter)
    _surface_particles_planar(b, mesh, dx, rng, jitter)
    _feature_particles(b, mesh, dx, rng, jitter)
    if len(mesh.singular):
        b.add(mesh.singular, SINGULAR, mesh.singular_vert)
    return geom, b, kind


def cylinder_workload(radius=0.5, height=1.0, segments=24, dx=0.08, jitter=0.3, seed=6, k=2,
                      move_mask=ALL_MOVING, name=None) -> Workload:
    """Upright cylinder (two closed rim loops of `segments` feature segments)
    filled like the batch's solids: volume lattice, per-facet-plane surface
    lattices, feature particles along the rims. No singular points."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mesh = M.cylinder(radius, height, segments)
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    _convex_volume_particles(b, mesh, dx, rng, jitter)
    _surface_particles_planar(b, mesh, dx, rng, jitter)
    _feature_particles(b, mesh, dx, rng, jitter)
    return _finish(name or f"cylinder{segments}_dx{dx:g}", [(geom, b)], move_mask, seed, {"dx": dx})


def split_geometry(wl: Workload, g: int) -> Workload:
    """Geometry g of a batch as a workload of its own (same particles, ids in
    batch order, owner and feature indices re-based)."""
    geo = wl.geoms[g]
    m = wl.gid == g
    b = _Builder()
    own = wl.owner[m].copy()
    tag = wl.tag[m]
    own[tag == SURFACE] -= geo.tri_begin
    own[tag == FEATURE] -= geo.feat_begin
    own[tag == SINGULAR] -= geo.vert_begin
    b.pos.append(wl.pos[m].astype(np.float64))
    b.tag.append(tag.copy())
    b.owner.append(own)
    nf = int(np.sum(tag == FEATURE))
    if nf:
        b.feat_seg.append(wl.feat_seg[geo.feat_begin:geo.feat_begin + nf] - geo.seg_begin)
        b.feat_u.append(wl.feat_u[geo.feat_begin:geo.feat_begin + nf].copy())
    single = Geometry(mesh=geo.mesh, dx=geo.dx, h=geo.h, k=geo.k, proj_radius=geo.proj_radius,
                      origin=geo.origin.copy(), inv_cell=geo.inv_cell, dims=geo.dims.copy(), csg=geo.csg)
    out = _finish(f"{wl.name}_g{g}", [(single, b)], wl.move_mask, wl.seed)
    out.pos = wl.pos[m].copy()     # keep the exact binary32 positions
    return out


def assembly_geometry(rng, n_target: float, jitter=0.3, k=2, mc_samples=1_000_000):
    """One Boolean assembly of 2-6 random boxes and cylinders (csg.random_assembly)
    with dx = (V / n_target)^(1/3) from its Monte Carlo volume V, filled like
    the other workloads: volume particles on a jittered (i+1/2)dx lattice at
    least dx/2 inside, surface particles on every part's faces where they lie
    on the assembly's boundary at least dx/2 from the other parts, feature
    particles along the clipped sharp edges, the surviving corners as
    singular points. Returns (Geometry, _Builder, description)."""
    parts, op, vol = C.random_assembly(rng, mc_samples)
    mesh, info, parts_P = C.combine(parts, op)
    dx = (vol / n_target) ** (1.0 / 3.0)
    geom = _make_geom(mesh, dx, k)
    geom.csg = info
    # the particle cells cover the solid (a difference lies inside part 0),
    # with a margin of one cell: the cell lookups clamp, so no stencil reaches out
    solid = parts if op == C.UNION else parts[:1]
    slo = np.min([p.vert.min(0) for p in solid], 0)
    shi = np.max([p.vert.max(0) for p in solid], 0)
    cell = float(f32((f32(2.0 * geom.h) / k) * (1.0 + 2.0 ** -8)))
    geom.origin, geom.inv_cell, geom.dims = particle_grid(slo, shi, geom.h, k, pad=cell)
    b = _Builder()
    lo, hi = mesh.bbox()
    axes = [np.arange(lo[a] + 0.5 * dx, hi[a], dx) for a in range(3)]
    for x in axes[0]:   # one x column at a time to bound memory
        g = np.stack(np.meshgrid([x], axes[1], axes[2], indexing="ij"), -1).reshape(-1, 3)
        g = g + rng.uniform(-jitter, jitter, g.shape) * dx
        b.add(g[C.inside_with_margin(op, parts_P, g, 0.5 * dx)], VOLUME)
    for q, part in enumerate(parts):
        bp = _Builder()
        _surface_particles_planar(bp, part, dx, rng, jitter)
        if not bp.pos:
            continue
        pts = np.concatenate(bp.pos, 0)
        own = np.concatenate(bp.owner)
        keep = C.on_boundary_with_margin(op, parts_P, q, pts, 0.5 * dx)
        b.add(pts[keep], SURFACE, own[keep] + info.part_tri_begin[q])
    _feature_particles(b, mesh, dx, rng, jitter)
    if len(mesh.singular):
        b.add(mesh.singular, SINGULAR, mesh.singular_vert)
    desc = {"op": "union" if op == C.UNION else "difference", "parts": len(parts),
            "kinds": ["box" if len(p.tri) == 12 else "cylinder" for p in parts], "volume": vol}
    return geom, b, desc


def batch_targets(n_geom=64, n_min=5e3, n_max=5e5, seed=4000):
    """The target particle counts of batch_workload's geometries (the first
    draw of each geometry's generator), without building them."""
    return [float(np.exp(np.random.Generator(np.random.PCG64(seed + g)).uniform(np.log(n_min), np.log(n_max))))
            for g in range(n_geom)]


def batch_workload(n_geom=64, n_min=5e3, n_max=5e5, seed=4000, jitter=0.3, k=2,
                   move_mask=ALL_MOVING, name=None, mc_samples=1_000_000, members=None) -> Workload:
    """A batch of independent Boolean assemblies relaxed together (section
    3.2.3 assemblies; assembly_geometry): geometry b uses PCG64 seed
    `seed + b` and a log-uniform target count in [n_min, n_max]. The
    geometries do not interact (each has its own cell grid and facets).
    members: build only these geometries of the batch (in the given order),
    each exactly as in the whole batch."""
    parts, descs, targets = [], [], []
    for g in (range(n_geom) if members is None else members):
        rng = np.random.Generator(np.random.PCG64(seed + g))
        n_t = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        geom, b, desc = assembly_geometry(rng, n_t, jitter, k, mc_samples)
        parts.append((geom, b))
        descs.append(desc)
        targets.append(n_t)
    meta = {"assemblies": descs, "targets": targets}
    if members is not None:
        meta["members"] = list(members)
    return _finish(name or (f"batch{n_geom}_seed{seed}" if members is None else
                            f"batch{n_geom}_seed{seed}_members{'_'.join(map(str, members))}"),
                   parts, move_mask, seed, meta)


def solid_batch_workload(n_geom=64, n_min=5e3, n_max=5e5, seed=4000, jitter=0.3, k=2,
                         move_mask=ALL_MOVING, name=None) -> Workload:
    """A batch of single convex solids (one box or cylinder per geometry)."""
    parts, kinds, targets = [], [], []
    for g in range(n_geom):
        rng = np.random.Generator(np.random.PCG64(seed + g))
        n_t = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        geom, b, kind = solid_geometry(rng, n_t, jitter, k)
        parts.append((geom, b))
        kinds.append(kind)
        targets.append(n_t)
    return _finish(name or f"solids{n_geom}_seed{seed}", parts, move_mask, seed,
                   {"kinds": kinds, "targets": targets})


# ---------------------------------------------------------------------------
# Extruded gear (24 teeth, central bore)
# ---------------------------------------------------------------------------

def _seg_dist2(p, a, b):
    """Squared distance of 2-D points p [..., 2] to segments a-b [..., 2]."""
    e = b - a
    w = p - a
    t = np.clip(np.sum(w * e, -1) / np.maximum(np.sum(e * e, -1), 1e-300), 0.0, 1.0)
    d = w - t[..., None] * e
    return np.sum(d * d, -1)


class _GearProfile:
    """The gear's 2-D outline and bore as polygons sampled at the same n
    angles (counter-clockwise), with a windowed distance query: the polygons
    are star-shaped about the axis, so the ray at angle theta crosses edge
    k = floor(theta n / 2 pi) and the closest edges are a few samples away."""

    def __init__(self, mesh: M.Mesh, n: int, rings: int):
        self.n, self.rings = n, rings
        top = (rings + 1) * n            # vertices of face 0 (z < 0) come first
        self.inner = mesh.vert[:n, :2].copy()
        self.outer = mesh.vert[rings * n: rings * n + n, :2].copy()
        assert top == len(mesh.vert) // 2
        r_out = np.linalg.norm(self.outer, axis=1)
        self.r_min_out = float(r_out.min())
        self.r_max_in = float(np.linalg.norm(self.inner, axis=1).max())

    def sector(self, p):
        th = np.mod(np.arctan2(p[:, 1], p[:, 0]), 2 * np.pi)
        return np.minimum((th * (self.n / (2 * np.pi))).astype(np.int64), self.n - 1)

    def _side(self, P, k, p):
        a, b = P[k], P[(k + 1) % self.n]
        return (b[:, 0] - a[:, 0]) * (p[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (p[:, 0] - a[:, 0])

    def _dist(self, P, k, p, W=4):
        best = np.full(len(p), np.inf)
        for o in range(-W, W + 1):
            kk = (k + o) % self.n
            best = np.minimum(best, _seg_dist2(p, P[kk], P[(kk + 1) % self.n]))
        return np.sqrt(best)

    def inside(self, p, margin):
        """2-D points strictly inside the annulus at least `margin` from both polygons."""
        rho = np.linalg.norm(p, axis=1)
        ok = (rho > self.r_max_in * 0.99) & (rho < 1.01 * float(np.linalg.norm(self.outer, axis=1).max()))
        deep = (rho > self.r_max_in + margin + 1e-5) & (rho < self.r_min_out * np.cos(np.pi / self.n) - margin - 1e-5)
        test = ok & ~deep
        idx = np.nonzero(test)[0]
        if len(idx):
            q = p[idx]
            k = self.sector(q)
            good = (self._side(self.outer, k, q) > 0) & (self._side(self.inner, k, q) < 0)
            good &= (self._dist(self.outer, k, q) >= margin) & (self._dist(self.inner, k, q) >= margin)
            test[idx] = good
        return deep | test


def _owner_by_candidates(mesh: M.Mesh, cand: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """First candidate facet (cand [P, C]) whose triangle contains each point
    (points on the facet's plane; barycentric coordinates >= -1e-12)."""
    out = np.full(len(pts), -1, np.int64)
    for c in range(cand.shape[1]):
        f = cand[:, c]
        A, B, C = (mesh.vert[mesh.tri[f, q]] for q in range(3))
        e0, e1, w = B - A, C - A, pts - A
        d00, d01, d11 = (np.einsum("ij,ij->i", x, y) for x, y in ((e0, e0), (e0, e1), (e1, e1)))
        d20, d21 = np.einsum("ij,ij->i", w, e0), np.einsum("ij,ij->i", w, e1)
        den = d00 * d11 - d01 * d01
        lb = (d11 * d20 - d01 * d21) / den
        lc = (d00 * d21 - d01 * d20) / den
        hit = (lb >= -1e-12) & (lc >= -1e-12) & (1 - lb - lc >= -1e-12) & (out < 0)
        out[hit] = f[hit]
    return out


def gear_workload(dx=0.004, jitter=0.3, seed=3, k=2, move_mask=ALL_MOVING, samples_per_period=60,
                  rings=35, name=None) -> Workload:
    """24-tooth extruded gear (meshes.gear: outer radius 1, root 0.85, bore
    0.2, thickness 0.3, ~207k facets) filled as in section 3.2:
      volume   (i+1/2)dx lattice jittered by U(+-jitter dx)^3, kept at least
               dx/2 inside every face;
      surface  top and bottom: jittered (i+1/2)dx lattice in the face plane at
               least dx/2 from the rims; walls: points at spacing ~dx in arc
               length around the rim times (b+1/2)dx in z, jittered in the
               wall, at least dx/2 from the rims and from the vertical sharp
               edges; owner = the facet containing the point;
      feature  spacing L/ceil(L/dx) along every sharp line, jittered along it;
      singular the 192 tooth corners on the rims."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mesh = M.gear(samples_per_period=samples_per_period, rings=rings)
    n = 24 * samples_per_period
    prof = _GearProfile(mesh, n, rings)
    geom = _make_geom(mesh, dx, k)
    b = _Builder()
    half = 0.15
    m = 0.5 * dx
    lo, hi = mesh.bbox()
    gx = np.arange(lo[0] + 0.5 * dx, hi[0], dx)
    gy = np.arange(lo[1] + 0.5 * dx, hi[1], dx)
    gz = np.arange(-half + 0.5 * dx, half, dx)
    # volume, one x column at a time to bound memory
    vol = []
    for x in gx:
        g = np.stack(np.meshgrid([x], gy, gz, indexing="ij"), -1).reshape(-1, 3)
        g = g + rng.uniform(-jitter, jitter, g.shape) * dx
        keep = (np.abs(g[:, 2]) <= half - m) & prof.inside(g[:, :2], m)
        vol.append(g[keep])
    b.add(np.concatenate(vol, 0), VOLUME)
    # top and bottom faces
    nf_face = rings * n * 2
    g2 = np.stack(np.meshgrid(gx, gy, indexing="ij"), -1).reshape(-1, 2)
    for face, z in enumerate((-half, half)):
        q = g2 + rng.uniform(-jitter, jitter, g2.shape) * dx
        q = q[prof.inside(q, m)]
        kq = prof.sector(q)
        r_in = np.linalg.norm(prof.inner[kq], axis=1)
        r_out = np.linalg.norm(prof.outer[kq], axis=1)
        s = (np.linalg.norm(q, axis=1) - r_in) / np.maximum(r_out - r_in, 1e-12)
        j0 = np.clip((s * rings).astype(np.int64), 0, rings - 1)
        cand = []
        for dj in (0, -1, 1):
            for dk in (0, -1, 1):
                jj = np.clip(j0 + dj, 0, rings - 1)
                kk = (kq + dk) % n
                base = face * nf_face + jj * (2 * n) + 2 * kk
                cand += [base, base + 1]
        cand = np.stack(cand, 1)
        pts = np.concatenate([q, np.full((len(q), 1), z)], 1)
        own = _owner_by_candidates(mesh, cand, pts)
        ok = own >= 0
        b.add(pts[ok], SURFACE, own[ok])
    # walls: bore (ring 0) and outline (ring `rings`)
    nf = 2 * nf_face
    corner = np.zeros(n, bool)
    corner[[kk for kk in range(n) if (kk % samples_per_period) in
            (0, samples_per_period // 3, samples_per_period // 2, (5 * samples_per_period) // 6)]] = True
    for wall, P in enumerate((prof.inner, prof.outer)):
        # points at spacing ~dx in arc length along the closed rim polygon
        a2, b2 = P, np.roll(P, -1, axis=0)
        L = np.linalg.norm(b2 - a2, axis=1)
        cum = np.concatenate([[0.0], np.cumsum(L)])
        m_arc = int(np.ceil(cum[-1] / dx))
        sp = cum[-1] / m_arc
        arc = np.repeat((np.arange(m_arc) + 0.5) * sp, len(gz))
        Z = np.tile(gz, m_arc)
        arc = np.mod(arc + rng.uniform(-jitter, jitter, len(arc)) * sp, cum[-1])
        Z = Z + rng.uniform(-jitter, jitter, len(Z)) * dx
        K = np.clip(np.searchsorted(cum, arc, side="right") - 1, 0, n - 1)
        U = (arc - cum[K]) / L[K]
        xy = a2[K] + U[:, None] * (b2[K] - a2[K])
        ok = np.abs(Z) <= half - m
        if wall == 1:   # stay clear of the vertical sharp edges at tooth corners
            for kc in (K, (K + 1) % n, (K - 1) % n, (K + 2) % n):
                ok &= ~(corner[kc] & (np.linalg.norm(xy - P[kc], axis=1) < m))
        K, xy, Z = K[ok], xy[ok], Z[ok]
        pts = np.concatenate([xy, Z[:, None]], 1)
        base = nf + wall * 2 * n + 2 * K
        own = _owner_by_candidates(mesh, np.stack([base, base + 1], 1), pts)
        good = own >= 0
        b.add(pts[good], SURFACE, own[good])
    _feature_particles(b, mesh, dx, rng, jitter)
    b.add(mesh.singular, SINGULAR, mesh.singular_vert)
    return _finish(name or f"gear24_dx{dx:g}", [(geom, b)], move_mask, seed, {"dx": dx})


def forced_reverts(wl: Workload, seed: int = 0, n_skin: int = 12, surface_every: int = 40) -> Workload:
    """The same single-geometry workload with particles placed where a step must
    revert (inputs for revert tests; no method arithmetic):
      * the first feature particle of every open line moved to 1e-7 of the
        line's start, where its neighbour along the line pushes it off the end;
      * every `surface_every`-th surface particle lifted off its facet along
        the facet normal by 1.5 times the projection radius;
      * `n_skin` volume particles put 1e-6 under the centroid of random facets,
        with every other particle within the support radius of that point that
        is not a deeper volume particle removed, so the volume pushes them out.
    """
    assert len(wl.geoms) == 1
    geo = wl.geoms[0]
    mesh = geo.mesh
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = wl.pos.astype(np.float64).copy()
    tag = wl.tag.copy()
    owner = wl.owner.copy()
    fs, fu = wl.feat_seg.copy(), wl.feat_u.copy()
    keep = np.ones(len(pos), bool)
    L = mesh.lines
    seg_line = np.zeros(L.n_seg, np.int64)
    for l in range(L.n_line):
        seg_line[L.line_seg_begin[l]:L.line_seg_begin[l + 1]] = l
    f = np.nonzero(tag == FEATURE)[0]
    if len(f):
        slot = owner[f]
        seg = fs[slot] - geo.seg_begin
        line = seg_line[seg]
        for l in range(L.n_line):
            if L.line_closed[l]:
                continue
            on = np.nonzero(line == l)[0]
            if len(on) == 0:
                continue
            first = on[np.lexsort((fu[slot[on]], seg[on]))[0]]
            s0 = int(L.line_seg_begin[l])
            a, b = L.seg_p[s0]
            u = 1e-7 * float(np.linalg.norm(b - a))
            fs[slot[first]], fu[slot[first]] = s0 + geo.seg_begin, u
            pos[f[first]] = a + (u / np.linalg.norm(b - a)) * (b - a)
    A, B, C = (mesh.vert[mesh.tri[:, q]] for q in range(3))
    nrm = np.cross(B - A, C - A)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    s = np.nonzero(tag == SURFACE)[0][::surface_every]
    pos[s] += 1.5 * float(geo.proj_radius) * nrm[owner[s] - geo.tri_begin]
    rc = 2.0 * float(geo.h)
    v = np.nonzero(tag == VOLUME)[0]
    for t in rng.choice(len(mesh.tri), size=min(n_skin, len(mesh.tri)), replace=False):
        c = (A[t] + B[t] + C[t]) / 3.0
        p = c - 1e-6 * nrm[t]
        d = np.linalg.norm(pos - p, axis=1)
        depth = (pos - c) @ nrm[t]
        near = keep & (d < rc)
        keep &= ~(near & ~((tag == VOLUME) & (depth < -0.3 * geo.dx)))
        k = v[np.argmin(np.where(keep[v], np.linalg.norm(pos[v] - p, axis=1), np.inf))]
        pos[k] = p
        keep[k] = True
    idx = np.nonzero(keep)[0]
    out = copy.copy(wl)
    out.pos = pos[idx].astype(np.float32)
    out.tag, out.owner, out.gid = tag[idx], owner[idx], wl.gid[idx]
    out.feat_seg, out.feat_u = fs, fu
    g2 = copy.copy(geo)
    g2.part_begin, g2.part_end = 0, len(idx)
    out.geoms = [g2]
    out.name = wl.name + "_forced_reverts"
    return out
