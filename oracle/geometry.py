"""Explicit-geometry primitives in FP64 (sections 3.1-3.2 of the paper).

  * facet frame: vertices A, B, C, unit outward normal n = (B-A)x(C-A)/|.|
  * projection of a point onto a facet plane along n and the barycentric
    coordinates of the foot point (section 3.2.1: the foot must lie inside
    the triangle; the paper tests this with cross products, here with the
    equivalent Gram-matrix solve)
  * exact point-triangle closest point by Voronoi regions (Ericson,
    Real-Time Collision Detection, 2005, section 5.1.5)
  * generalised winding number from facet solid angles (Van Oosterom and
    Strackee, 1983) -> inside/outside sign for the signed distance
"""
import numpy as np


def facet_frames(vert: np.ndarray, tri: np.ndarray):
    A = vert[tri[:, 0]]
    B = vert[tri[:, 1]]
    C = vert[tri[:, 2]]
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n, axis=1)[:, None]
    return A, B, C, n


def barycentric(p, A, B, C):
    """Barycentric coordinates (la, lb, lc) of points p in triangles (A, B, C)
    (all broadcastable [..., 3]), from the 2x2 Gram system of the edge vectors."""
    e0 = B - A
    e1 = C - A
    v = p - A
    d00 = np.sum(e0 * e0, -1)
    d01 = np.sum(e0 * e1, -1)
    d11 = np.sum(e1 * e1, -1)
    d20 = np.sum(v * e0, -1)
    d21 = np.sum(v * e1, -1)
    den = d00 * d11 - d01 * d01
    lb = (d11 * d20 - d01 * d21) / den
    lc = (d00 * d21 - d01 * d20) / den
    return 1.0 - lb - lc, lb, lc


def closest_point_triangle(p, a, b, c):
    """Closest point of triangle abc to p (single point, FP64), Voronoi-region method."""
    ab = b - a
    ac = c - a
    ap = p - a
    d1 = ab @ ap
    d2 = ac @ ap
    if d1 <= 0 and d2 <= 0:
        return a
    bp = p - b
    d3 = ab @ bp
    d4 = ac @ bp
    if d3 >= 0 and d4 <= d3:
        return b
    vc = d1 * d4 - d3 * d2
    if vc <= 0 and d1 >= 0 and d3 <= 0:
        return a + (d1 / (d1 - d3)) * ab
    cp = p - c
    d5 = ab @ cp
    d6 = ac @ cp
    if d6 >= 0 and d5 <= d6:
        return c
    vb = d5 * d2 - d1 * d6
    if vb <= 0 and d2 >= 0 and d6 <= 0:
        return a + (d2 / (d2 - d6)) * ac
    va = d3 * d6 - d5 * d4
    if va <= 0 and (d4 - d3) >= 0 and (d5 - d6) >= 0:
        return b + ((d4 - d3) / ((d4 - d3) + (d5 - d6))) * (c - b)
    denom = 1.0 / (va + vb + vc)
    return a + ab * (vb * denom) + ac * (vc * denom)


def unsigned_distance(p, vert, tri) -> float:
    """min over all facets of the exact point-triangle distance."""
    best = np.inf
    for t in range(len(tri)):
        q = closest_point_triangle(p, vert[tri[t, 0]], vert[tri[t, 1]], vert[tri[t, 2]])
        best = min(best, float(np.linalg.norm(p - q)))
    return best


def winding_number(p: np.ndarray, vert, tri) -> np.ndarray:
    """Generalised winding number of a closed outward mesh at points p [N, 3]:
    sum of facet solid angles / (4 pi); ~1 inside, ~0 outside."""
    p = np.atleast_2d(p)
    out = np.zeros(len(p))
    A, B, C, _ = facet_frames(vert, tri)
    for s in range(0, len(p), 512):
        q = p[s:s + 512, None, :]
        a, b, c = A[None] - q, B[None] - q, C[None] - q
        la = np.linalg.norm(a, axis=-1)
        lb = np.linalg.norm(b, axis=-1)
        lc = np.linalg.norm(c, axis=-1)
        num = np.einsum("ntk,ntk->nt", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("ntk,ntk->nt", a, b) * lc
               + np.einsum("ntk,ntk->nt", a, c) * lb + np.einsum("ntk,ntk->nt", b, c) * la)
        out[s:s + 512] = np.sum(2.0 * np.arctan2(num, den), axis=1) / (4.0 * np.pi)
    return out


def signed_distance(p: np.ndarray, vert, tri) -> np.ndarray:
    """Signed distance to a closed mesh, negative inside (winding number > 1/2)."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    wn = winding_number(p, vert, tri)
    d = np.array([unsigned_distance(q, vert, tri) for q in p])
    return np.where(wn > 0.5, -d, d)


def unsigned_distance_many(p: np.ndarray, vert, tri, chunk=1 << 22) -> np.ndarray:
    """Vectorised form of unsigned_distance for points [P, 3]: the same
    Voronoi-region cases evaluated for every (point, facet) pair."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    A, B, C, _ = facet_frames(vert, tri)
    out = np.full(len(p), np.inf)
    step = max(1, chunk // max(len(tri), 1))
    for s in range(0, len(p), step):
        q = p[s:s + step, None, :]
        a, b, c = A[None], B[None], C[None]
        ab, ac = b - a, c - a
        ap, bp, cp = q - a, q - b, q - c
        d1 = np.sum(ab * ap, -1); d2 = np.sum(ac * ap, -1)
        d3 = np.sum(ab * bp, -1); d4 = np.sum(ac * bp, -1)
        d5 = np.sum(ab * cp, -1); d6 = np.sum(ac * cp, -1)
        va = d3 * d6 - d5 * d4
        vb = d5 * d2 - d1 * d6
        vc = d1 * d4 - d3 * d2
        with np.errstate(divide="ignore", invalid="ignore"):
            t_ab = d1 / (d1 - d3)
            t_ac = d2 / (d2 - d6)
            t_bc = (d4 - d3) / ((d4 - d3) + (d5 - d6))
            den = 1.0 / (va + vb + vc)
        r_a = (d1 <= 0) & (d2 <= 0)
        r_b = ~r_a & (d3 >= 0) & (d4 <= d3)
        r_ab = ~r_a & ~r_b & (vc <= 0) & (d1 >= 0) & (d3 <= 0)
        r_c = ~r_a & ~r_b & ~r_ab & (d6 >= 0) & (d5 <= d6)
        r_ac = ~r_a & ~r_b & ~r_ab & ~r_c & (vb <= 0) & (d2 >= 0) & (d6 <= 0)
        r_bc = ~r_a & ~r_b & ~r_ab & ~r_c & ~r_ac & (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0)
        face = ~(r_a | r_b | r_ab | r_c | r_ac | r_bc)
        cl = np.where(face[..., None], a + ab * (vb * den)[..., None] + ac * (vc * den)[..., None], 0.0)
        cl = np.where(r_a[..., None], a, cl)
        cl = np.where(r_b[..., None], b, cl)
        cl = np.where(r_c[..., None], c, cl)
        cl = np.where(r_ab[..., None], a + t_ab[..., None] * ab, cl)
        cl = np.where(r_ac[..., None], a + t_ac[..., None] * ac, cl)
        cl = np.where(r_bc[..., None], b + t_bc[..., None] * (c - b), cl)
        out[s:s + step] = np.min(np.linalg.norm(q - cl, axis=-1), axis=1)
    return out


def signed_distance_many(p: np.ndarray, vert, tri) -> np.ndarray:
    """signed_distance for many points (vectorised distance, same sign rule)."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    wn = winding_number(p, vert, tri)
    d = unsigned_distance_many(p, vert, tri)
    return np.where(wn > 0.5, -d, d)
