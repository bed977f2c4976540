"""Facet registration on a uniform grid and the sparse storage of the
registered cells (sections 3.1.1 and 3.1.3, Eq. 9-10).

TEST INFRASTRUCTURE ONLY, like the rest of this package: plain Python loops
and numpy, FP64.

  subdivide   recursive midpoint subdivision with virtual points (section
              3.1.1): an edge whose extent along some axis exceeds the cell
              edge is split at its midpoint (a + b) * 0.5; the midpoints of the
              other edges are virtual. A triangle with no split edge (its
              box fits one cell along every axis) is a leaf. Children keep the
              orientation: three split edges give the 4 corner-and-centre
              triangles; two give the corner where they meet plus the rest of
              the triangle cut along the diagonal from the far end of the
              unsplit edge (reading: the paper's figure shows 3 children, not
              which diagonal); one gives 2 triangles through the opposite
              vertex.
  register    for each leaf, the cells its box reaches (widened by pad; at most
              two per axis for a leaf) that pass the closed separating-axis
              test against the cell's box widened by pad (generate.tri_box_overlap);
              the pairs (cell, facet) of all leaves, unique, sorted.
  morton      Eq. 9: the bits of the cell coordinates interleaved, x lowest,
              then y, then z.
  hash        Eq. 10: (p1 x + p2 y + p3 z) mod H with the paper's primes, in
              64-bit unsigned arithmetic (reading: the paper gives no width).
  sparse      C_compact: the registered cells in Morton order with begin and
              length of their facets in the (morton, facet)-sorted list; the
              hash table: C_compact reordered by (hash, morton), H_begin and
              H_length per hash value (H = the number of registered cells,
              reading: the paper names H_size without a value).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .generate import tri_box_overlap

P1, P2, P3 = 738560931, 19349663, 83492791
MAX_LEVELS = 48


def _needs_split(p, q, cell):
    return max(abs(q[0] - p[0]), abs(q[1] - p[1]), abs(q[2] - p[2])) > cell


def _mid(p, q):
    return tuple((p[k] + q[k]) * 0.5 for k in range(3))


def children(a, b, c, cell):
    """The children of triangle (a, b, c), or None for a leaf."""
    s = (_needs_split(a, b, cell), _needs_split(b, c, cell), _needs_split(c, a, cell))
    n = sum(s)
    if n == 0:
        return None
    if n == 3:
        mab, mbc, mca = _mid(a, b), _mid(b, c), _mid(c, a)
        return [(a, mab, mca), (mab, b, mbc), (mca, mbc, c), (mab, mbc, mca)]
    # rotate so that the cyclic order is (u, v, w) with edge (u, v) the unsplit
    # one (two split) or the split one (one split)
    verts = (a, b, c)
    if n == 2:
        r = s.index(False)
        u, v, w = verts[r], verts[(r + 1) % 3], verts[(r + 2) % 3]
        mvw, mwu = _mid(v, w), _mid(w, u)
        return [(mvw, w, mwu), (u, v, mvw), (u, mvw, mwu)]
    r = s.index(True)
    u, v, w = verts[r], verts[(r + 1) % 3], verts[(r + 2) % 3]
    muv = _mid(u, v)
    return [(u, muv, w), (muv, v, w)]


def subdivide(vert, tri, cell, facets=None):
    """Leaves [(facet, a, b, c)] of every facet (or of `facets`), per facet in
    depth-first order."""
    out = []
    ids = range(len(tri)) if facets is None else facets
    for t in ids:
        root = tuple(tuple(float(x) for x in vert[v]) for v in tri[t])
        stack = [(root, 0)]
        while stack:
            (a, b, c), lvl = stack.pop()
            ch = children(a, b, c, cell)
            if ch is None:
                out.append((int(t), a, b, c))
                continue
            if lvl + 1 >= MAX_LEVELS:
                raise ValueError("subdivision deeper than MAX_LEVELS")
            for x in reversed(ch):
                stack.append((x, lvl + 1))
    return out


def leaf_cells(a, b, c, origin, cell, dims, pad):
    """Cells (x, y, z) of the grid met by one leaf."""
    P = np.array([a, b, c], np.float64)
    inv = 1.0 / cell
    lo = [max(0, int(np.floor((P[:, q].min() - pad - origin[q]) * inv))) for q in range(3)]
    hi = [min(dims[q] - 1, int(np.floor((P[:, q].max() + pad - origin[q]) * inv))) for q in range(3)]
    cells = [(x, y, z) for z in range(lo[2], hi[2] + 1) for y in range(lo[1], hi[1] + 1)
             for x in range(lo[0], hi[0] + 1)]
    if not cells:
        return []
    C = np.array(cells, np.int64)
    cen = origin + (C.astype(np.float64) + 0.5) * cell
    hw = np.full(cen.shape, 0.5 * cell + pad)
    ok = tri_box_overlap(cen, hw, P[0][None], P[1][None], P[2][None])
    return [cells[i] for i in np.nonzero(ok)[0]]


def register(vert, tri, origin, cell, dims, pad, facets=None):
    """Unique (x, y, z, facet) rows [M, 4] of the registration, sorted by
    (z, y, x, facet)."""
    origin = np.asarray(origin, np.float64)
    rows = set()
    for t, a, b, c in subdivide(vert, tri, cell, facets):
        for x, y, z in leaf_cells(a, b, c, origin, cell, dims, pad):
            rows.add((x, y, z, t))
    if not rows:
        return np.zeros((0, 4), np.int64)
    R = np.array(sorted(rows, key=lambda r: (r[2], r[1], r[0], r[3])), np.int64)
    return R


def dense_csr(rows, dims):
    """Facet lists per cell of a dense grid (x fastest): start [ncell + 1], facets."""
    ncell = int(np.prod(dims))
    key = (rows[:, 2] * dims[1] + rows[:, 1]) * dims[0] + rows[:, 0]
    start = np.searchsorted(key, np.arange(ncell + 1), side="left").astype(np.int64)
    return start, rows[:, 3].astype(np.int64)


def morton(x, y, z, bits=21):
    """Eq. 9 for non-negative integer coordinates below 2^bits."""
    code = 0
    for i in range(bits):
        code |= ((int(x) >> i) & 1) << (3 * i)
        code |= ((int(y) >> i) & 1) << (3 * i + 1)
        code |= ((int(z) >> i) & 1) << (3 * i + 2)
    return code


def hash_value(x, y, z, size):
    """Eq. 10 in 64-bit unsigned arithmetic (products and sum modulo 2^64)."""
    return ((P1 * int(x) + P2 * int(y) + P3 * int(z)) & ((1 << 64) - 1)) % int(size)


@dataclass
class Sparse:
    morton: np.ndarray    # [C] uint64, ascending: C_compact's cells
    begin: np.ndarray     # [C] first facet of the cell in `facets`
    length: np.ndarray    # [C]
    facets: np.ndarray    # [M] facets sorted by (morton, facet)
    size: int             # H_size
    order: np.ndarray     # [C] C_compact indices sorted by (hash, morton)
    h_begin: np.ndarray   # [H] first position in `order` of each hash value
    h_length: np.ndarray  # [H]
    xyz: np.ndarray       # [C, 3] cell coordinates of C_compact


def sparse(rows, size=None):
    """The compact list and the hash table of a registration."""
    codes = np.array([morton(x, y, z) for x, y, z, _ in rows], dtype=np.uint64)
    o = np.lexsort((rows[:, 3], codes))
    codes, rows = codes[o], rows[o]
    head = np.ones(len(codes), bool)
    head[1:] = codes[1:] != codes[:-1]
    cb = np.nonzero(head)[0]
    length = np.diff(np.append(cb, len(codes)))
    C = len(cb)
    H = int(size if size is not None else max(C, 1))
    xyz = rows[cb, :3]
    hv = np.array([hash_value(x, y, z, H) for x, y, z in xyz], np.int64)
    order = np.lexsort((codes[cb], hv))
    h_length = np.bincount(hv, minlength=H).astype(np.int64)
    h_begin = np.concatenate([[0], np.cumsum(h_length)[:-1]]).astype(np.int64)
    return Sparse(codes[cb], cb.astype(np.int64), length.astype(np.int64), rows[:, 3].copy(), H, order.astype(np.int64),
                  h_begin, h_length, xyz)


def lookup(sp: Sparse, x, y, z):
    """The facets registered in cell (x, y, z), through the hash table."""
    h = hash_value(x, y, z, sp.size)
    code = morton(x, y, z)
    for q in range(sp.h_begin[h], sp.h_begin[h] + sp.h_length[h]):
        c = sp.order[q]
        if int(sp.morton[c]) == code:
            return sp.facets[sp.begin[c]:sp.begin[c] + sp.length[c]]
    return np.zeros(0, np.int64)
