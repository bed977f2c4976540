"""Synthetic triangle meshes and their sharp-feature polylines.

These stand in for the STL models of the paper (the gears, tire, sphere and
assemblies of its experiments), which are not available. Every mesh is a
closed, outward-oriented triangle surface given as FP64 vertices and int32
facet corner indices; feature polylines (sharp edges) and singular points are
produced by construction from the same parametrisation, not extracted.

This module is shared by the oracle and the GPU path as an input generator
only: it holds geometry construction, no step of the relaxation method.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class FeatureLines:
    """Polylines along sharp edges.

    line_seg_begin[l] .. line_seg_begin[l+1] are the segments of line l, in
    order along the line; segment s runs from seg_p[s, 0] to seg_p[s, 1] and
    consecutive segments of a line share endpoints. line_closed[l] = 1 for a
    loop (the last segment ends where the first begins).
    """
    line_seg_begin: np.ndarray  # int32 [n_line + 1]
    seg_p: np.ndarray           # float64 [n_seg, 2, 3]
    line_closed: np.ndarray     # uint8 [n_line]
    seg_vert: np.ndarray = None  # int32 [n_seg, 2]: mesh vertex at each segment end (-1: none)

    @property
    def n_line(self) -> int:
        return int(self.line_closed.shape[0])

    @property
    def n_seg(self) -> int:
        return int(self.seg_p.shape[0])

    @staticmethod
    def empty() -> "FeatureLines":
        return FeatureLines(np.zeros(1, np.int32), np.zeros((0, 2, 3)), np.zeros(0, np.uint8),
                            np.zeros((0, 2), np.int32))

    @staticmethod
    def from_polylines(polys, closed, vert_ids=None) -> "FeatureLines":
        """Lines through the given points; vert_ids[l][k] = mesh vertex of point k of line l."""
        begins = [0]
        segs, sv = [], []
        for li, pts in enumerate(polys):
            pts = np.asarray(pts, np.float64)
            ids = np.full(len(pts), -1) if vert_ids is None else np.asarray(vert_ids[li])
            for k, (a, b) in enumerate(zip(pts[:-1], pts[1:])):
                segs.append((a, b))
                sv.append((ids[k], ids[k + 1]))
            begins.append(len(segs))
        seg_p = np.array(segs, np.float64).reshape(-1, 2, 3)
        return FeatureLines(np.array(begins, np.int32), seg_p, np.array(closed, np.uint8),
                            np.array(sv, np.int32).reshape(-1, 2))


@dataclass
class Mesh:
    vert: np.ndarray   # float64 [nv, 3]
    tri: np.ndarray    # int32 [nt, 3], counter-clockwise seen from outside
    lines: FeatureLines = field(default_factory=FeatureLines.empty)
    singular: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))  # float64 [ns, 3]
    singular_vert: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))  # vertex of each

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    def bbox(self):
        return self.vert.min(0), self.vert.max(0)


def _orient_outward(vert, tri, inside_point):
    """Flip facets whose corner order gives a normal pointing at inside_point."""
    a, b, c = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a - inside_point) < 0
    tri = tri.copy()
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def cube(lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> Mesh:
    """Axis-aligned box as 12 facets (two per face), 12 feature edges, 8 corners."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    corners = np.array([[(hi if (c >> a) & 1 else lo)[a] for a in range(3)] for c in range(8)])
    quads = []
    for axis in range(3):
        u, v = [a for a in range(3) if a != axis]
        for side in (0, 1):
            ids = [c for c in range(8) if ((c >> axis) & 1) == side]
            # order the four corners of the face around its boundary
            ids.sort(key=lambda c: (((c >> u) & 1), ((c >> v) & 1)))
            q = [ids[0], ids[1], ids[3], ids[2]]
            quads.append(q)
    tri = []
    for q in quads:
        tri.append([q[0], q[1], q[2]])
        tri.append([q[0], q[2], q[3]])
    tri = _orient_outward(corners, np.array(tri, np.int32), (lo + hi) / 2)
    edges = [(a, b) for a in range(8) for b in range(a + 1, 8) if bin(a ^ b).count("1") == 1]
    lines = FeatureLines.from_polylines([[corners[a], corners[b]] for a, b in edges], [0] * len(edges),
                                        [[a, b] for a, b in edges])
    return Mesh(corners, tri.astype(np.int32), lines, corners.copy(), np.arange(8, dtype=np.int32))


def tetrahedron() -> Mesh:
    """Regular tetrahedron of edge 1, its 6 edges as features and 4 corners."""
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, np.sqrt(3) / 2, 0.0],
                  [0.5, np.sqrt(3) / 6, np.sqrt(2.0 / 3.0)]])
    tri = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], np.int32)
    tri = _orient_outward(v, tri, v.mean(0))
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    lines = FeatureLines.from_polylines([[v[a], v[b]] for a, b in edges], [0] * len(edges),
                                        [[a, b] for a, b in edges])
    return Mesh(v, tri, lines, v.copy(), np.arange(4, dtype=np.int32))


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    """Icosahedron subdivided `level` times, vertices on the sphere: 20*4^level facets."""
    t = (1.0 + np.sqrt(5.0)) / 2.0
    v = [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
         [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]]
    v = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
         [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
         [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = nf
    vert = np.array(v) * radius
    tri = _orient_outward(vert, np.array(f, np.int32), np.zeros(3))
    return Mesh(vert, tri.astype(np.int32))


def gear(teeth=24, r_tip=1.0, r_root=0.85, r_bore=0.2, half_thick=0.15,
         samples_per_period=60, rings=35) -> Mesh:
    """Extruded gear with trapezoidal teeth and a central bore.

    Outline radius per tooth period (360/teeth degrees): root for 1/3 of the
    period, a linear flank up over 1/6, the tip for 1/3, a flank down over 1/6.
    The outline and the bore are sampled at the same angles; top and bottom
    faces are triangulated as `rings` annular strips between them; side walls
    are one strip of skinny facets in z. Sharp features: the outline and bore
    rims at both faces (closed loops broken at tooth corners) and the vertical
    edges at tooth corners.
    """
    n = teeth * samples_per_period
    theta = np.arange(n) * (2 * np.pi / n)
    ph = (np.arange(n) % samples_per_period) / samples_per_period  # phase in [0,1)
    r = np.empty(n)
    r[ph < 1 / 3] = r_root
    m = (ph >= 1 / 3) & (ph < 1 / 2)
    r[m] = r_root + (r_tip - r_root) * (ph[m] - 1 / 3) * 6
    m = (ph >= 1 / 2) & (ph < 5 / 6)
    r[m] = r_tip
    m = ph >= 5 / 6
    r[m] = r_tip - (r_tip - r_root) * (ph[m] - 5 / 6) * 6
    outer = np.stack([r * np.cos(theta), r * np.sin(theta)], 1)
    inner = np.stack([r_bore * np.cos(theta), r_bore * np.sin(theta)], 1)
    s = np.linspace(0.0, 1.0, rings + 1)
    ring_xy = inner[None] * (1 - s[:, None, None]) + outer[None] * s[:, None, None]  # [rings+1, n, 2]
    verts = []
    for z in (-half_thick, half_thick):
        zz = np.full((rings + 1, n, 1), z)
        verts.append(np.concatenate([ring_xy, zz], 2).reshape(-1, 3))
    vert = np.concatenate(verts, 0)
    base_top = (rings + 1) * n

    def vid(face, ring, k):
        return face * base_top + ring * n + (k % n)

    tri = []
    for face in (0, 1):
        for ring in range(rings):
            for k in range(n):
                a, b = vid(face, ring, k), vid(face, ring, k + 1)
                c, d = vid(face, ring + 1, k), vid(face, ring + 1, k + 1)
                tri.append([a, b, d])
                tri.append([a, d, c])
    for ring in (0, rings):
        for k in range(n):
            a, b = vid(0, ring, k), vid(0, ring, k + 1)
            c, d = vid(1, ring, k), vid(1, ring, k + 1)
            tri.append([a, b, d])
            tri.append([a, d, c])
    tri = np.array(tri, np.int32)
    # orientation: top/bottom by z sign, walls radially (outer wall outward, bore inward)
    A, B, C = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    nrm = np.cross(B - A, C - A)
    cen = (A + B + C) / 3
    nf = 2 * rings * n * 2
    want = np.zeros_like(nrm)
    want[: nf // 2, 2] = -1
    want[nf // 2: nf, 2] = 1
    radial = np.concatenate([cen[nf:, :2], np.zeros((len(tri) - nf, 1))], 1)
    wall_bore = np.arange(len(tri) - nf) < n * 2
    radial[wall_bore] *= -1
    want[nf:] = radial
    flip = np.einsum("ij,ij->i", nrm, want) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    # features: corners of the outline are where the phase hits 0, 1/3, 1/2, 5/6
    corner_k = [k for k in range(n) if (k % samples_per_period) in
                (0, samples_per_period // 3, samples_per_period // 2, (5 * samples_per_period) // 6)]
    polys, closed = [], []
    singular, sing_vert, vids = [], [], []
    for face_of_z, z in enumerate((-half_thick, half_thick)):
        pts = np.concatenate([outer, np.full((n, 1), z)], 1)
        for ci in range(len(corner_k)):
            k0, k1 = corner_k[ci], corner_k[(ci + 1) % len(corner_k)]
            ks = list(range(k0, k1 + 1)) if k1 > k0 else list(range(k0, n)) + list(range(0, k1 + 1))
            polys.append(pts[np.array(ks) % n])
            vids.append([vid(face_of_z, rings, kk) for kk in ks])
            closed.append(0)
        for k in corner_k:
            singular.append(pts[k])
            sing_vert.append(vid(face_of_z, rings, k))
        bore = np.concatenate([inner, np.full((n, 1), z)], 1)
        polys.append(np.concatenate([bore, bore[:1]], 0))
        vids.append([vid(face_of_z, 0, kk) for kk in range(n)] + [vid(face_of_z, 0, 0)])
        closed.append(1)
    for k in corner_k:
        p0 = np.array([outer[k, 0], outer[k, 1], -half_thick])
        p1 = np.array([outer[k, 0], outer[k, 1], half_thick])
        polys.append(np.stack([p0, p1]))
        vids.append([vid(0, rings, k), vid(1, rings, k)])
        closed.append(0)
    lines = FeatureLines.from_polylines(polys, closed, vids)
    return Mesh(vert, tri, lines, np.array(singular), np.array(sing_vert, np.int32))


def cylinder(radius=0.5, height=1.0, segments=64) -> Mesh:
    """Closed cylinder along z centred at the origin: fan caps and a side wall of
    `segments` quads (4*segments facets); features are the two rim loops."""
    th = np.arange(segments) * (2 * np.pi / segments)
    ring = np.stack([radius * np.cos(th), radius * np.sin(th)], 1)
    zb, zt = -height / 2, height / 2
    vert = np.concatenate([np.concatenate([ring, np.full((segments, 1), zb)], 1),
                           np.concatenate([ring, np.full((segments, 1), zt)], 1),
                           [[0.0, 0.0, zb], [0.0, 0.0, zt]]], 0)
    cb, ct = 2 * segments, 2 * segments + 1
    tri = []
    for k in range(segments):
        a, b = k, (k + 1) % segments
        tri.append([cb, b, a])                         # bottom cap
        tri.append([ct, segments + a, segments + b])   # top cap
        tri.append([a, b, segments + b])               # side
        tri.append([a, segments + b, segments + a])
    tri = _orient_outward(vert, np.array(tri, np.int32), np.zeros(3))
    loops = [np.concatenate([vert[:segments], vert[:1]], 0),
             np.concatenate([vert[segments:2 * segments], vert[segments:segments + 1]], 0)]
    lines = FeatureLines.from_polylines(loops, [1, 1], [list(range(segments)) + [0],
                                                        list(range(segments, 2 * segments)) + [segments]])
    return Mesh(vert, tri.astype(np.int32), lines, np.zeros((0, 3)))


def transformed(mesh: Mesh, R: np.ndarray, t: np.ndarray) -> Mesh:
    """Rigid motion x -> R x + t of a mesh, its feature lines and singular points."""
    seg = mesh.lines.seg_p @ R.T + t
    lines = FeatureLines(mesh.lines.line_seg_begin.copy(), seg, mesh.lines.line_closed.copy(),
                         None if mesh.lines.seg_vert is None else mesh.lines.seg_vert.copy())
    sing = mesh.singular @ R.T + t if len(mesh.singular) else mesh.singular.copy()
    return Mesh(mesh.vert @ R.T + t, mesh.tri.copy(), lines, sing, mesh.singular_vert.copy())
