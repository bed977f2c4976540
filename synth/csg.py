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
    e = b - a
    s0 = P[:, 0] * a[0] + P[:, 1] * a[1] + P[:, 2] * a[2] - P[:, 3]
    s1 = P[:, 0] * e[0] + P[:, 1] * e[1] + P[:, 2] * e[2]
    par = s1 == 0.0
    if np.any(par & (s0 >= 0.0)):
        return None
    t = -s0[~par] / s1[~par]
    up = s1[~par] > 0
    hi = t[up].min() if up.any() else np.inf
    lo = t[~up].max() if (~up).any() else -np.inf
    return (float(lo), float(hi)) if lo < hi else None


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


def _tri_pair_segments(A, B):
    """Segments where facets of convex part A meet facets of part B (both
    [n, 3, 3] vertex arrays, outward counter-clockwise): for every pair of
    facets (f, g) whose corners of f lie strictly on both sides of g's plane,
    the chord of f in that plane (its first two crossing points in edge order
    (0,1), (1,2), (2,0); a corner on the plane counts as a crossing), clipped
    to g. Returns (p, q, f, g) tuples."""
    nB = np.cross(B[:, 1] - B[:, 0], B[:, 2] - B[:, 0])
    nB /= np.linalg.norm(nB, axis=1, keepdims=True)
    dB = np.einsum("ij,ij->i", nB, B[:, 0])
    scale = max(np.ptp(A.reshape(-1, 3), 0).max(), np.ptp(B.reshape(-1, 3), 0).max())
    eps = 1e-12 * scale
    S = np.einsum("fkc,gc->fgk", A, nB) - dB[None, :, None]          # [nA, nB, 3]
    fi, gi = np.nonzero((S.max(2) > eps) & (S.min(2) < -eps))
    if len(fi) == 0:
        return []
    s = S[fi, gi]                                                     # [K, 3]
    F = A[fi]                                                         # [K, 3, 3]
    pts = np.zeros((len(fi), 3, 3))
    ok = np.zeros((len(fi), 3), bool)
    for e, (i0, i1) in enumerate(((0, 1), (1, 2), (2, 0))):
        a, b = s[:, i0], s[:, i1]
        cross = ((a > eps) & (b < -eps)) | ((a < -eps) & (b > eps))
        on = np.abs(a) <= eps
        t = np.where(cross, a / np.where(cross, a - b, 1.0), 0.0)
        pts[:, e] = np.where(cross[:, None], F[:, i0] + t[:, None] * (F[:, i1] - F[:, i0]), F[:, i0])
        ok[:, e] = cross | on
    two = ok.sum(1) >= 2
    first = np.argmax(ok, 1)
    ok2 = ok.copy()
    ok2[np.arange(len(fi)), first] = False
    second = np.argmax(ok2, 1)
    P0 = pts[np.arange(len(fi)), first]
    Q0 = pts[np.arange(len(fi)), second]
    G = B[gi]
    n = nB[gi]
    lo = np.zeros(len(fi))
    hi = np.ones(len(fi))
    for u, v in ((0, 1), (1, 2), (2, 0)):
        m = np.cross(n, G[:, v] - G[:, u])                                # into g
        s0 = np.einsum("ij,ij->i", m, P0 - G[:, u])
        s1 = np.einsum("ij,ij->i", m, Q0 - P0)
        par = np.abs(s1) < 1e-300
        t = -s0 / np.where(par, 1.0, s1)
        lo = np.where(~par & (s1 > 0), np.maximum(lo, t), lo)
        hi = np.where(~par & (s1 < 0), np.minimum(hi, t), hi)
        hi = np.where(par & (s0 < 0), -1.0, hi)
    keep = two & (hi - lo > 1e-12)
    out = []
    for k in np.nonzero(keep)[0]:
        p, q = P0[k], Q0[k]
        out.append((p + lo[k] * (q - p), p + hi[k] * (q - p), int(fi[k]), int(gi[k])))
    return out


def _on_boundary_intervals(op, parts_P, j, k, a, b, eps=1e-9):
    """Parameter intervals of segment a-b, which lies on the surfaces of parts
    j < k, that lie on the assembly's boundary."""
    iv = [(0.0, 1.0)]
    if op == DIFFERENCE and j >= 1:
        c = _inside_interval(parts_P[0], a, b)   # two cut parts meet inside part 0 only
        iv = [] if c is None else [(max(0.0, c[0]), min(1.0, c[1]))]
    for l, P in enumerate(parts_P):
        if l in (j, k) or (op == DIFFERENCE and l == 0):
            continue
        iv = _subtract(iv, _inside_interval(P, a, b))
    return [(s, e) for s, e in iv if e - s > eps]


def _weld(points, tol):
    """Labels [n] merging points closer than tol (union-find over KD-tree pairs)."""
    from scipy.spatial import cKDTree
    pts = np.asarray(points, np.float64).reshape(-1, 3)
    parent = np.arange(len(pts))

    def root(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    if len(pts):
        for a, b in sorted(cKDTree(pts).query_pairs(tol)):
            ra, rb = root(a), root(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    return np.array([root(i) for i in range(len(pts))], np.int64)


def _chain(segments, tol):
    """Polylines through segments that share end points (within tol): open
    chains between points of degree other than two, then the loops."""
    if not segments:
        return [], []
    ends = np.array([[a, b] for a, b in segments], np.float64).reshape(-1, 3)
    lab = _weld(ends, tol)
    pts = {int(l): ends[i] for i, l in enumerate(lab)}
    adj = {}
    for k in range(len(segments)):
        i, j = int(lab[2 * k]), int(lab[2 * k + 1])
        if i == j:
            continue
        adj.setdefault(i, []).append(j)
        adj.setdefault(j, []).append(i)
    used = set()
    polys, closed = [], []

    def walk(s, t):
        line = [s, t]
        used.add((min(s, t), max(s, t)))
        while len(adj[line[-1]]) == 2 and line[-1] != s:
            nxt = [x for x in adj[line[-1]] if (min(line[-1], x), max(line[-1], x)) not in used]
            if not nxt:
                break
            used.add((min(line[-1], nxt[0]), max(line[-1], nxt[0])))
            line.append(nxt[0])
        return line

    for s in sorted(n for n, nb in adj.items() if len(nb) != 2):
        for t in sorted(adj[s]):
            if (min(s, t), max(s, t)) not in used:
                polys.append([pts[i] for i in walk(s, t)])
                closed.append(0)
    for s in sorted(adj):
        for t in sorted(adj[s]):
            if (min(s, t), max(s, t)) not in used:
                line = walk(s, t)
                polys.append([pts[i] for i in line])
                closed.append(1 if line[-1] == s else 0)
    return polys, closed


def _in_tri(T, x, tol):
    e0, e1, w = T[1] - T[0], T[2] - T[0], x - T[0]
    d00, d01, d11 = e0 @ e0, e0 @ e1, e1 @ e1
    d20, d21 = w @ e0, w @ e1
    den = d00 * d11 - d01 * d01
    v = (d11 * d20 - d01 * d21) / den
    u = (d00 * d21 - d01 * d20) / den
    return v >= -tol and u >= -tol and v + u <= 1 + tol


def _face_on_boundary(op, parts_P, q, T, m, d, delta):
    """Does facet T of part q lie on the assembly's boundary next to the
    segment through m along d (a probe point a little into T on either side)?"""
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n /= np.linalg.norm(n)
    u = np.cross(n, d)
    for sgn in (1.0, -1.0):
        x = m + sgn * delta * u
        if _in_tri(T, x, 1e-9) and on_boundary_with_margin(op, parts_P, q, x[None], 1e-3 * delta)[0]:
            return True
    return False


def intersection_lines(op, parts, parts_P):
    """The curves where two parts' surfaces meet on the assembly's boundary
    and form a crease (the two faces next to the curve both lie on the
    boundary; a part face buried behind a coplanar face of the other part
    gives none), as polylines: sharp edges of the assembly that are edges of
    no part."""
    segs = []
    scale = max(np.ptp(p.vert, 0).max() for p in parts)
    delta = 1e-6 * scale
    for j in range(len(parts)):
        Aj = parts[j].vert[parts[j].tri]
        for k in range(j + 1, len(parts)):
            Ak = parts[k].vert[parts[k].tri]
            for a, b, fi, gi in _tri_pair_segments(Aj, Ak):
                for t0, t1 in _on_boundary_intervals(op, parts_P, j, k, a, b):
                    pa, pb = a + t0 * (b - a), a + t1 * (b - a)
                    d = (pb - pa) / np.linalg.norm(pb - pa)
                    m = 0.5 * (pa + pb)
                    if _face_on_boundary(op, parts_P, j, Aj[fi], m, d, delta) and \
                            _face_on_boundary(op, parts_P, k, Ak[gi], m, d, delta):
                        segs.append((pa, pb))
    return _chain(segs, 1e-9 * scale)


def combine(parts, op, with_curves=True):
    """One facet list for all parts (each part's facets in a contiguous range)."""
    vb = np.concatenate([[0], np.cumsum([len(p.vert) for p in parts])]).astype(np.int32)
    tb = np.concatenate([[0], np.cumsum([len(p.tri) for p in parts])]).astype(np.int32)
    vert = np.concatenate([p.vert for p in parts], 0)
    tri = np.concatenate([p.tri + vb[k] for k, p in enumerate(parts)], 0).astype(np.int32)
    parts_P = [planes(p) for p in parts]
    lines, sing, sing_v = clip_lines(op, parts, parts_P, vb)
    if with_curves:
        lines, sing, sing_v = _add_curves(op, parts, parts_P, lines, sing, sing_v)
    mesh = M.Mesh(vert, tri, lines, sing, sing_v)
    return mesh, CSG(op, tb, vb), parts_P


def _add_curves(op, parts, parts_P, lines, sing, sing_v):
    """The parts' clipped sharp edges together with the intersection curves.
    Every end of an open line becomes a singular point (with its mesh vertex
    when it is one, -1 at a clip or crossing point), and lines are cut at the
    singular points they pass through, so that every line runs between
    singular points or is a loop without one."""
    polys, closed, vids = [], [], []
    for l in range(lines.n_line):
        s0, s1 = int(lines.line_seg_begin[l]), int(lines.line_seg_begin[l + 1])
        polys.append([lines.seg_p[s0, 0]] + [lines.seg_p[s, 1] for s in range(s0, s1)])
        vids.append([int(lines.seg_vert[s0, 0])] + [int(lines.seg_vert[s, 1]) for s in range(s0, s1)])
        closed.append(int(lines.line_closed[l]))
    cp, cc = intersection_lines(op, parts, parts_P)
    for pts, c in zip(cp, cc):
        polys.append(pts)
        vids.append([-1] * len(pts))
        closed.append(c)
    tol = 1e-9 * max(np.ptp(p.vert, 0).max() for p in parts)
    cand, cand_v = [np.asarray(p) for p in sing], [int(v) for v in sing_v]
    for pts, ids, c in zip(polys, vids, closed):
        if not c:
            cand += [np.asarray(pts[0]), np.asarray(pts[-1])]
            cand_v += [ids[0], ids[-1]]
    lab = _weld(cand, tol) if cand else np.zeros(0, np.int64)
    out_s, out_v, seen = [], [], {}
    for i, l in enumerate(lab):
        if int(l) not in seen:
            seen[int(l)] = len(out_s)
            out_s.append(cand[i])
            out_v.append(cand_v[i])
        elif out_v[seen[int(l)]] < 0 <= cand_v[i]:
            out_v[seen[int(l)]] = cand_v[i]
    S = np.array(out_s, np.float64).reshape(-1, 3)
    from scipy.spatial import cKDTree
    tree = cKDTree(S) if len(S) else None

    def is_sing(p):
        return tree is not None and tree.query(np.asarray(p), distance_upper_bound=tol)[0] <= tol

    new_p, new_c, new_v = [], [], []
    for pts, ids, c in zip(polys, vids, closed):
        cut = [k for k in range(len(pts) - (1 if c else 0)) if is_sing(pts[k])]
        if c and cut:   # a loop through singular points: open lines between them
            r = cut[0]
            ring, rid = pts[r:-1] + pts[:r + 1], ids[r:-1] + ids[:r + 1]
            cut = [k for k in range(len(ring)) if is_sing(ring[k])]
            pts, ids, c = ring, rid, 0
        if not c:
            cut = sorted(set([0] + [k for k in cut if 0 < k < len(pts) - 1] + [len(pts) - 1]))
            for a, b in zip(cut[:-1], cut[1:]):
                new_p.append(pts[a:b + 1])
                new_v.append(ids[a:b + 1])
                new_c.append(0)
        else:
            new_p.append(pts)
            new_v.append(ids)
            new_c.append(1)
    new_lines = M.FeatureLines.from_polylines(new_p, new_c, new_v) if new_p else M.FeatureLines.empty()
    return new_lines, S, np.array(out_v, np.int32)


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
