"""Feature extraction and feature-line particles (section 3.2.2), in FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the product path never imports it.

  feature edges   every mesh edge (vertex pair, smaller index first) with its
                  facets; an edge with other than two facets is a feature
                  edge; an edge between two facets is one iff the angle
                  between their outward unit normals exceeds the threshold,
                  i.e. n1 . n2 < cos_threshold. (The paper compares the
                  dihedral angle with a threshold; the reading takes the
                  angle between the facet normals, 180 degrees minus the
                  interior dihedral angle.) Unit normals: cross product of
                  the edge vectors B - A and C - A divided by its length; sums
                  of three products left to right.
  singular points vertices on one feature edge or on more than two.
  feature lines   maximal chains of feature edges: from every singular vertex
                  along each of its feature edges until the next singular
                  vertex (each line kept once, from the end whose (vertex,
                  next vertex) pair is smaller); the remaining feature edges
                  form loops, each started at its smallest vertex towards the
                  smaller of that vertex's two neighbours. Lines are listed
                  in the order of their (start vertex, second vertex), loops
                  after the lines, ordered the same way.
  particles       per line of length L, n = max(1, ceil(L / dx)) equal arc-
                  length steps L/n: open lines get the n - 1 interior points
                  (their ends are singular points), loops get n points
                  starting at their first vertex; a singular particle sits on
                  every singular vertex.
"""
import math

import numpy as np


def _dot(u, v):
    return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]


def unit_normals(vert, tri):
    out = np.empty((len(tri), 3))
    for t, (a, b, c) in enumerate(tri):
        n = np.cross(vert[b] - vert[a], vert[c] - vert[a])
        out[t] = n / math.sqrt(_dot(n, n))
    return out


def feature_edges(vert, tri, cos_threshold):
    """Sorted list of feature edges (u, v), u < v."""
    edges = {}
    for t, f in enumerate(tri):
        for u, v in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
            edges.setdefault((min(u, v), max(u, v)), []).append(t)
    n = unit_normals(vert, tri)
    out = []
    for key, fs in edges.items():
        if len(fs) != 2 or _dot(n[fs[0]], n[fs[1]]) < cos_threshold:
            out.append((int(key[0]), int(key[1])))
    return sorted(out)


def singular_vertices(fe):
    deg = {}
    for u, v in fe:
        deg[u] = deg.get(u, 0) + 1
        deg[v] = deg.get(v, 0) + 1
    return sorted(x for x, d in deg.items() if d != 2)


def feature_lines(fe):
    """(lines, closed): lines as vertex lists."""
    nb = {}
    for u, v in fe:
        nb.setdefault(u, []).append(v)
        nb.setdefault(v, []).append(u)
    for k in nb:
        nb[k].sort()
    sing = set(x for x, l in nb.items() if len(l) != 2)
    used = set()
    opened = []
    for s in sorted(sing):
        for w in nb[s]:
            line = [s, w]
            prev, cur = s, w
            while cur not in sing:
                a, b = nb[cur]
                nxt = b if a == prev else a
                prev, cur = cur, nxt
                line.append(cur)
            start = (line[0], line[1])
            end = (line[-1], line[-2])
            if start <= end:
                for p, q in zip(line[:-1], line[1:]):
                    used.add((min(p, q), max(p, q)))
                if start < end or line not in opened:
                    opened.append(line)
    loops = []
    rest = [e for e in fe if e not in used]
    seen = set()
    for u, v in sorted(rest):
        if (u, v) in seen:
            continue
        # walk the loop containing (u, v)
        loop = [u, v]
        prev, cur = u, v
        while cur != u:
            a, b = nb[cur]
            nxt = b if a == prev else a
            prev, cur = cur, nxt
            loop.append(cur)
        loop = loop[:-1]
        for p, q in zip(loop, loop[1:] + loop[:1]):
            seen.add((min(p, q), max(p, q)))
        m = loop.index(min(loop))
        loop = loop[m:] + loop[:m]
        if loop[-1] < loop[1]:
            loop = [loop[0]] + loop[1:][::-1]
        loops.append(loop)
    opened.sort(key=lambda l: (l[0], l[1]))
    loops.sort(key=lambda l: (l[0], l[1]))
    return opened + loops, [0] * len(opened) + [1] * len(loops)


def line_particles(vert, line, closed, dx):
    """Points at equal arc-length steps along a polyline (see the module note)."""
    pts = [vert[v] for v in line] + ([vert[line[0]]] if closed else [])
    seg = [math.sqrt(_dot(q - p, q - p)) for p, q in zip(pts[:-1], pts[1:])]
    L = 0.0
    for s in seg:
        L += s
    n = max(1, math.ceil(L / dx))
    ks = range(0, n) if closed else range(1, n)
    out = []
    for k in ks:
        target = k * (L / n)
        acc, i = 0.0, 0
        while i < len(seg) - 1 and acc + seg[i] < target:
            acc += seg[i]
            i += 1
        t = (target - acc) / seg[i]
        out.append(pts[i] + t * (pts[i + 1] - pts[i]))
    return out


def extract(vert, tri, cos_threshold, dx):
    """(feature edges, singular vertices, lines, closed, feature particles [P, 3],
    singular particles [S, 3])."""
    vert = np.asarray(vert, np.float64)
    tri = np.asarray(tri)
    fe = feature_edges(vert, tri, cos_threshold)
    sing = singular_vertices(fe)
    lines, closed = feature_lines(fe)
    parts = []
    for l, c in zip(lines, closed):
        parts += line_particles(vert, l, c, dx)
    return fe, sing, lines, closed, np.array(parts).reshape(-1, 3), vert[sing].reshape(-1, 3)
