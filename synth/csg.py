"""Boolean assemblies of convex parts: the inputs of the batched workload.

An assembly is the union of 2-6 parts, or part 0 minus the union of the
others (section 3.2.3 combines solids by Boolean operations; the parts here
are random boxes and 64-segment cylinders). This module builds the inputs
only, with FP64 plane tests on the convex parts: the combined facet list, the
parts' sharp edges clipped to the assembly's boundary, and the particle
seeds on and inside it. It holds no step of the relaxation method.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import meshes as M

UNION, DIFFERENCE = 1, 2


@dataclass
class CSG:
    op: int                      # UNION or DIFFERENCE (part 0 minus the others)
    part_tri_begin: np.ndarray   # int32 [n_part + 1]: facets of part k in the combined mesh
    part_vert_begin: np.ndarray  # int32 [n_part + 1]

    @property
    def n_part(self) -> int:
        return len(self.part_tri_begin) - 1


def planes(mesh: M.Mesh) -> np.ndarray:
    """(n, d) of every facet of a convex outward mesh, n unit: inside iff n.x - d < 0 for all."""
    A, B, C = (mesh.vert[mesh.tri[:, q]] for q in range(3))
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return np.concatenate([n, np.einsum("ij,ij->i", n, A)[:, None]], 1)


def plane_sd(P: np.ndarray, x: np.ndarray) -> np.ndarray:
    """max over the planes of n.x - d: negative inside; its magnitude bounds the
    distance to the part's surface from below inside and outside."""
    return np.max(np.asarray(x, np.float64) @ P[:, :3].T - P[:, 3], axis=1)


def inside_with_margin(op, parts_P, x, margin):
    """Points at least `margin` inside the assembly (by the plane bounds)."""
    sd = np.stack([plane_sd(P, x) for P in parts_P], 1)
    if op == UNION:
        return sd.min(1) <= -margin
    return (sd[:, 0] <= -margin) & ((sd[:, 1:].min(1) if sd.shape[1] > 1 else np.inf) >= margin)


def on_boundary_with_margin(op, parts_P, k, x, margin):
    """Points of part k's surface that lie on the assembly's boundary at least
    `margin` away from every other part."""
    keep = np.ones(len(x), bool)
    for j, P in enumerate(parts_P):
        if j == k:
            continue
        sd = plane_sd(P, x)
        if op == DIFFERENCE and k > 0 and j == 0:
            keep &= sd <= -margin       # a cut face is on the boundary where it lies inside part 0
        else:
            keep &= sd >= margin
    return keep


def _inside_interval(P, a, b):
    """Open parameter interval (lo, hi) of a + t (b - a) strictly inside the part."""
    lo, hi = -np.inf, np.inf
    e = b - a
    for n0, n1, n2, d in P:
        s0 = n0 * a[0] + n1 * a[1] + n2 * a[2] - d
        s1 = n0 * e[0] + n1 * e[1] + n2 * e[2]
        if s1 == 0.0:
            if s0 >= 0.0:
                return None
            continue
        t = -s0 / s1
        if s1 > 0:
            hi = min(hi, t)
        else:
            lo = max(lo, t)
    return (lo, hi) if lo < hi else None


def _subtract(iv, cut):
    out = []
    for s, e in iv:
        if cut is None or cut[1] <= s or cut[0] >= e:
            out.append((s, e))
            continue
        if cut[0] > s:
            out.append((s, cut[0]))
        if cut[1] < e:
            out.append((cut[1], e))
    return out


def _surviving(op, parts_P, k, a, b, eps=1e-9):
    """Parameter intervals of segment a-b (an edge of part k) on the assembly's boundary."""
    iv = [(0.0, 1.0)]
    if op == DIFFERENCE and k > 0:
        c = _inside_interval(parts_P[0], a, b)
        iv = [] if c is None else [(max(0.0, c[0]), min(1.0, c[1]))]
    for j, P in enumerate(parts_P):
        if j == k or (op == DIFFERENCE and j == 0):
            continue
        iv = _subtract(iv, _inside_interval(P, a, b))
    return [(s, e) for s, e in iv if e - s > eps]


def clip_lines(op, parts, parts_P, vert_begin):
    """The parts' feature lines restricted to the assembly's boundary, as one
    FeatureLines (segment end vertices re-based to the combined mesh, -1 at
    clip points) and the surviving corners (singular points)."""
    polys, closed, vids = [], [], []
    for k, mesh in enumerate(parts):
        L = mesh.lines
        for l in range(L.n_line):
            s0, s1 = int(L.line_seg_begin[l]), int(L.line_seg_begin[l + 1])
            pieces = []    # [points, vertex ids, starts at the line's start, reaches the line's end]
            cur = None     # the piece being extended; cur[3]: it reaches the end of the last segment seen
            for s in range(s0, s1):
                a, b = L.seg_p[s]
                va, vb = (int(v) + vert_begin[k] if v >= 0 else -1 for v in L.seg_vert[s])
                iv = _surviving(op, parts_P, k, a, b)
                if not iv and cur is not None:
                    cur[3] = False
                for t0, t1 in iv:
                    pa = a + t0 * (b - a) if t0 > 0.0 else a
                    pb = a + t1 * (b - a) if t1 < 1.0 else b
                    ia = va if t0 == 0.0 else -1
                    ib = vb if t1 == 1.0 else -1
                    if cur is not None and cur[3] and t0 == 0.0:
                        cur[0].append(pb)
                        cur[1].append(ib)
                    else:
                        if cur is not None:
                            cur[3] = False
                            pieces.append(cur)
                        cur = [[pa, pb], [ia, ib], s == s0 and t0 == 0.0, True]
                    cur[3] = t1 == 1.0
            if cur is not None:
                pieces.append(cur)
            if L.line_closed[l] and len(pieces) == 1 and pieces[0][2] and pieces[0][3] \
                    and len(pieces[0][0]) == s1 - s0 + 1:
                polys.append(pieces[0][0][:-1] + [pieces[0][0][0]])   # the whole loop survives
                vids.append(pieces[0][1][:-1] + [pieces[0][1][0]])
                closed.append(1)
                continue
            if L.line_closed[l] and len(pieces) > 1 and pieces[0][2] and pieces[-1][3]:
                # the loop's last piece runs on into its first one
                last = pieces.pop()
                first = pieces[0]
                pieces[0] = [last[0] + first[0][1:], last[1] + first[1][1:], last[2], first[3]]
            for pts, ids, _, _ in pieces:
                polys.append(pts)
                vids.append(ids)
                closed.append(0)
    lines = M.FeatureLines.from_polylines(polys, closed, vids) if polys else M.FeatureLines.empty()
    sing, sing_v = [], []
    for k, mesh in enumerate(parts):
        for c, v in zip(mesh.singular, mesh.singular_vert):
            if on_boundary_with_margin(op, parts_P, k, c[None], 1e-9)[0]:
                sing.append(c)
                sing_v.append(int(v) + vert_begin[k])
    return lines, np.array(sing, np.float64).reshape(-1, 3), np.array(sing_v, np.int32)


def combine(parts, op):
    """One facet list for all parts (each part's facets in a contiguous range)."""
    vb = np.concatenate([[0], np.cumsum([len(p.vert) for p in parts])]).astype(np.int32)
    tb = np.concatenate([[0], np.cumsum([len(p.tri) for p in parts])]).astype(np.int32)
    vert = np.concatenate([p.vert for p in parts], 0)
    tri = np.concatenate([p.tri + vb[k] for k, p in enumerate(parts)], 0).astype(np.int32)
    parts_P = [planes(p) for p in parts]
    lines, sing, sing_v = clip_lines(op, parts, parts_P, vb)
    mesh = M.Mesh(vert, tri, lines, sing, sing_v)
    return mesh, CSG(op, tb, vb), parts_P


def random_part(rng) -> M.Mesh:
    """A box (edges U(0.1, 1)) or a 64-segment cylinder (diameter and height
    U(0.1, 1)), each with probability 1/2, randomly rotated."""
    if rng.uniform() < 0.5:
        e = rng.uniform(0.1, 1.0, 3)
        mesh = M.cube(-e / 2, e / 2)
    else:
        dia, hgt = rng.uniform(0.1, 1.0, 2)
        mesh = M.cylinder(dia / 2, hgt, 64)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    return mesh, R


def random_assembly(rng, mc_samples=1_000_000):
    """2-6 parts: part 0 at the origin, the others centred U(-0.3, 0.3)^3;
    union or difference with probability 1/2; redrawn while the result holds
    less than 10 % of part 0's volume. Returns (parts, op, volume by
    seeded Monte Carlo)."""
    while True:
        m = int(rng.integers(2, 7))
        parts = []
        for k in range(m):
            mesh, R = random_part(rng)
            t = np.zeros(3) if k == 0 else rng.uniform(-0.3, 0.3, 3)
            parts.append(M.transformed(mesh, R, t))
        op = UNION if rng.uniform() < 0.5 else DIFFERENCE
        parts_P = [planes(p) for p in parts]
        lo = np.min([p.vert.min(0) for p in (parts if op == UNION else parts[:1])], 0)
        hi = np.max([p.vert.max(0) for p in (parts if op == UNION else parts[:1])], 0)
        x = rng.uniform(lo, hi, size=(mc_samples, 3))
        frac = np.mean(inside_with_margin(op, parts_P, x, 0.0))
        vol = float(frac * np.prod(hi - lo))
        x0 = rng.uniform(parts[0].vert.min(0), parts[0].vert.max(0), size=(mc_samples // 4, 3))
        v0 = float(np.mean(plane_sd(parts_P[0], x0) < 0) * np.prod(parts[0].vert.max(0) - parts[0].vert.min(0)))
        if vol >= 0.1 * v0:
            return parts, op, vol
