"""Particle generation front end (sections 3.1.1, 3.1.2 and 3.2.1), in FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the product path never imports it.

On a uniform background grid of edge dx (cell (i, j, k) spans
origin + [i, i+1) dx, ...; its centre is origin + (i + 1/2) dx, each
coordinate computed as origin + (index + 0.5) * dx in FP64):

  surface cells  cells whose closed box meets a facet, by the separating-axis
                 triangle-box test (the 3 box normals, the facet normal and the
                 9 products of box axes with facet edges). The paper subdivides
                 facets until their bounding box is at most one cell before
                 testing; a cell meets the facet iff it meets one of its
                 sub-triangles, so the set of surface cells is the same.
  internal cells non-surface cells whose centre is inside by ray casting: the
                 number of facets crossed by the vertical segment from below
                 the mesh up to the centre is odd.
  particles      a volume particle at the centre of every internal cell; a
                 surface particle at the projection of every surface cell's
                 centre along the normal of the nearest facet (smallest
                 |plane distance|, ties to the lowest facet index) among the
                 facets meeting the cell whose projection falls inside the
                 facet (all barycentric coordinates >= 0); a cell with none is
                 discarded.

Readings (the paper does not say): the ray crossing uses a fill rule so that a
vertical line through a shared edge or vertex of the xy-projection is counted
once: a facet's projection is made counter-clockwise, a point strictly inside
counts, and a point on an edge counts iff that edge points down in y, or
along -x when horizontal, each edge function being evaluated for the edge's
endpoints in a fixed (lexicographic) order and negated for the other
direction, so that two facets sharing an edge see exactly opposite values.
Facets with a zero-area projection (vertical) are not crossed. A crossing at
height z toggles every cell whose centre is strictly above z. "Distance" in
the mapping is the plane distance along the facet normal (the projection of
section 3.3.3 without the radius limit).
"""
import numpy as np

EXTERNAL, INTERNAL, SURFACE = 0, 1, 2
VOLUME_TAG, SURFACE_TAG = 3, 2


def centres(origin, dx, n):
    return origin + (np.arange(n, dtype=np.float64) + 0.5) * dx


def tri_box_overlap(c, hw, a, b, cc):
    """Separating-axis test of triangles (a, b, cc) [..., 3] against boxes with
    centres c and half-widths hw [..., 3] (closed: touching counts)."""
    v0, v1, v2 = a - c, b - c, cc - c
    e = [v1 - v0, v2 - v1, v0 - v2]
    ok = np.ones(np.broadcast(v0[..., 0], c[..., 0]).shape, bool)
    # the 9 axes e_k x f_j
    for f in e:
        for k in range(3):
            axis = np.zeros(f.shape)
            k1, k2 = (k + 1) % 3, (k + 2) % 3
            axis[..., k1] = -f[..., k2]
            axis[..., k2] = f[..., k1]
            p0 = np.sum(v0 * axis, -1)
            p1 = np.sum(v1 * axis, -1)
            p2 = np.sum(v2 * axis, -1)
            r = np.sum(hw * np.abs(axis), -1)
            ok &= ~((np.minimum(np.minimum(p0, p1), p2) > r) | (np.maximum(np.maximum(p0, p1), p2) < -r))
    # the box normals
    for k in range(3):
        lo = np.minimum(np.minimum(v0[..., k], v1[..., k]), v2[..., k])
        hi = np.maximum(np.maximum(v0[..., k], v1[..., k]), v2[..., k])
        ok &= ~((lo > hw[..., k]) | (hi < -hw[..., k]))
    # the facet normal
    n = np.cross(e[0], e[1])
    d = np.sum(n * v0, -1)
    r = np.sum(hw * np.abs(n), -1)
    ok &= ~(np.abs(d) > r)
    return ok


def _edge_fn(pa, pb, px, py):
    """Edge function of the directed edge pa -> pb at (px, py), evaluated with
    the endpoints in lexicographic order and negated for the other direction."""
    swap = (pa[..., 0] > pb[..., 0]) | ((pa[..., 0] == pb[..., 0]) & (pa[..., 1] > pb[..., 1]))
    u = np.where(swap[..., None], pb, pa)
    w = np.where(swap[..., None], pa, pb)
    e = (w[..., 0] - u[..., 0]) * (py - u[..., 1]) - (w[..., 1] - u[..., 1]) * (px - u[..., 0])
    return np.where(swap, -e, e)


def _owns_edge(pa, pb):
    dxe = pb[..., 0] - pa[..., 0]
    dye = pb[..., 1] - pa[..., 1]
    return (dye < 0) | ((dye == 0) & (dxe < 0))


def column_crossings(A, B, C, px, py):
    """For facets (A, B, C) [T, 3] and one column point (px, py): mask of
    facets crossed by the vertical line and the crossing heights."""
    P = [A[:, :2], B[:, :2], C[:, :2]]
    area = (P[1][:, 0] - P[0][:, 0]) * (P[2][:, 1] - P[0][:, 1]) - (P[1][:, 1] - P[0][:, 1]) * (P[2][:, 0] - P[0][:, 0])
    cw = area < 0
    Q1 = np.where(cw[:, None], P[2], P[1])
    Q2 = np.where(cw[:, None], P[1], P[2])
    Q = [P[0], Q1, Q2]
    inside = area != 0
    for i in range(3):
        a, b = Q[i], Q[(i + 1) % 3]
        e = _edge_fn(a, b, px, py)
        inside &= (e > 0) | ((e == 0) & _owns_edge(a, b))
    # height of the facet plane over (px, py): barycentric in the projection
    with np.errstate(divide="ignore", invalid="ignore"):
        l1 = ((px - P[0][:, 0]) * (P[2][:, 1] - P[0][:, 1]) - (py - P[0][:, 1]) * (P[2][:, 0] - P[0][:, 0])) / area
        l2 = ((P[1][:, 0] - P[0][:, 0]) * (py - P[0][:, 1]) - (P[1][:, 1] - P[0][:, 1]) * (px - P[0][:, 0])) / area
        z = A[:, 2] + l1 * (B[:, 2] - A[:, 2]) + l2 * (C[:, 2] - A[:, 2])
    return inside, z


def classify(vert, tri, dx, origin, dims):
    """Cell classes [nz, ny, nx] (EXTERNAL / INTERNAL / SURFACE)."""
    origin = np.asarray(origin, np.float64)
    nx, ny, nz = (int(v) for v in dims)
    A, B, C = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    cls = np.zeros((nz, ny, nx), np.uint8)
    hw = np.full(3, 0.5 * dx)
    cx, cy, cz = centres(origin[0], dx, nx), centres(origin[1], dx, ny), centres(origin[2], dx, nz)
    # surface cells: every facet against the cells of its bounding box
    for t in range(len(tri)):
        lo = np.minimum(np.minimum(A[t], B[t]), C[t])
        hi = np.maximum(np.maximum(A[t], B[t]), C[t])
        i0 = np.clip(np.floor((lo - origin) / dx).astype(int) - 1, 0, np.array([nx, ny, nz]) - 1)
        i1 = np.clip(np.floor((hi - origin) / dx).astype(int) + 1, 0, np.array([nx, ny, nz]) - 1)
        gx, gy, gz = np.meshgrid(np.arange(i0[0], i1[0] + 1), np.arange(i0[1], i1[1] + 1),
                                 np.arange(i0[2], i1[2] + 1), indexing="ij")
        cen = np.stack([cx[gx.ravel()], cy[gy.ravel()], cz[gz.ravel()]], 1)
        hit = tri_box_overlap(cen, hw, A[t], B[t], C[t])
        cls[gz.ravel()[hit], gy.ravel()[hit], gx.ravel()[hit]] = SURFACE
    # ray parity per column
    for j in range(ny):
        for i in range(nx):
            inside, z = column_crossings(A, B, C, cx[i], cy[j])
            par = np.zeros(nz, np.int64)
            for zz in z[inside]:
                par += cz > zz
            col = cls[:, j, i]
            cls[:, j, i] = np.where((col != SURFACE) & (par % 2 == 1), INTERNAL, col)
    return cls


def _dot(u, v):
    return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]


def surface_particle(vert, tri, facets, c):
    """Projection of the cell centre c onto the nearest facet of `facets`
    (plane distance, ties to the lowest index) whose foot lies inside it;
    (None, -1) if none. Sums of three products are taken left to right."""
    best, bt, bp = np.inf, -1, None
    for t in sorted(facets):
        a, b, cc = vert[tri[t, 0]], vert[tri[t, 1]], vert[tri[t, 2]]
        n = np.cross(b - a, cc - a)
        n = n / np.sqrt(_dot(n, n))
        d = _dot(c - a, n)
        p = c - d * n
        e0, e1, v = b - a, cc - a, p - a
        d00, d01, d11 = _dot(e0, e0), _dot(e0, e1), _dot(e1, e1)
        d20, d21 = _dot(v, e0), _dot(v, e1)
        den = d00 * d11 - d01 * d01
        lb = (d11 * d20 - d01 * d21) / den
        lc = (d00 * d21 - d01 * d20) / den
        if min(1.0 - lb - lc, lb, lc) >= 0.0 and abs(d) < best:
            best, bt, bp = abs(d), t, p
    return bp, bt


def generate(vert, tri, dx, origin, dims):
    """(cls, pos [P, 3] float64, tag [P], owner [P]) in cell order (z, y, x)."""
    vert = np.asarray(vert, np.float64)
    tri = np.asarray(tri)
    origin = np.asarray(origin, np.float64)
    nx, ny, nz = (int(v) for v in dims)
    cls = classify(vert, tri, dx, origin, dims)
    cx, cy, cz = centres(origin[0], dx, nx), centres(origin[1], dx, ny), centres(origin[2], dx, nz)
    A, B, C = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    hw = np.full(3, 0.5 * dx)
    pos, tag, owner = [], [], []
    for k, j, i in zip(*np.nonzero(cls)):
        c = np.array([cx[i], cy[j], cz[k]])
        if cls[k, j, i] == INTERNAL:
            pos.append(c); tag.append(VOLUME_TAG); owner.append(-1)
            continue
        hit = np.flatnonzero(tri_box_overlap(c[None], hw[None], A, B, C))
        p, t = surface_particle(vert, tri, hit, c)
        if t >= 0:
            pos.append(p); tag.append(SURFACE_TAG); owner.append(t)
    return cls, np.array(pos).reshape(-1, 3), np.array(tag, np.int32), np.array(owner, np.int32)


UNION, INTERSECTION, DIFFERENCE = 0, 1, 2


def boolean(cls_a, cls_b, op):
    """Cell classes of a Boolean combination of two solids classified on the
    same grid (section 3.2.3). Reading: the paper combines the solids' cell
    sets as set operations on their internal (volume-particle) cells; surface
    cells are kept where the combined surface can pass:
      union         I = Ai | Bi;          S = (As & ~Bi) | (Bs & ~Ai)
      intersection  I = Ai & Bi;          S = (As & (Bi | Bs)) | (Bs & (Ai | As))
      difference    I = Ai & ~(Bi | Bs);  S = (As & ~Bi) | (Bs & (Ai | As))
    with S taken outside I."""
    ai, as_ = cls_a == INTERNAL, cls_a == SURFACE
    bi, bs = cls_b == INTERNAL, cls_b == SURFACE
    if op == UNION:
        i = ai | bi
        s = (as_ & ~bi) | (bs & ~ai)
    elif op == INTERSECTION:
        i = ai & bi
        s = (as_ & (bi | bs)) | (bs & (ai | as_))
    elif op == DIFFERENCE:
        i = ai & ~(bi | bs)
        s = (as_ & ~bi) | (bs & (ai | as_))
    else:
        raise ValueError(op)
    out = np.zeros_like(cls_a)
    out[s & ~i] = SURFACE
    out[i] = INTERNAL
    return out
