"""One relaxation iteration (section 3.3.2-3.3.4, Algorithm 1), in FP64.

Order of the iteration, following Algorithm 1:
  1. accelerations of all moving particles (Eq. 15, force.py)
  2. time step: the paper takes it from Eq. 24 of its reference [Ji et al.
     2021], which is not reproduced. Reading (parity unpinned):
         dt = 0.25 sqrt(h / amax),  amax = max over moving particles of |a_i|
     per geometry, so that dt^2 = (h/16)/amax.
  3. velocity reset to zero, then v = a dt (Eq. 22 with v_n = 0), and
     dr = v dt = a dt^2 (Eq. 23): the particle with the largest acceleration
     moves exactly h/16.
  4. displacement restricted to the geometry (Eq. 24-25). Eq. 24-25 as printed
     project the position onto a plane through the origin; the reading is that
     the displacement is projected onto the plane of the particle's own facet:
         surface:  dr <- dr - (dr . n) n   (n = unit normal of the owner facet)
     Feature-line particles move along their line (the paper places them,
     section 3.2.2, but does not spell out their motion; reading, parity
     unpinned): du = dr . t with t the unit tangent of the owner segment, then
     the arc-length coordinate u advances by du along the polyline, carrying
     into the neighbouring segments of the same line; leaving an open line
     reverts the move, a closed line wraps.
     Volume particles move by dr. Singular and fixed particles never move.
  5. projection (section 3.3.3): a surface particle at y = x + dr is projected
     along the normal onto every facet; a projection is accepted if its foot
     lies inside the facet (all barycentric coordinates >= 0) and |d| <= R;
     the accepted facet with the smallest |d| wins (ties: lowest facet index)
     and becomes the new owner; if none is accepted the particle returns to
     its previous position. The paper searches the 27 grid cells around the
     particle; with facets registered conservatively in cells of edge >= R
     that search sees every facet whose accepted foot point is within R, so
     the brute-force search over all facets here gives the same result.
     Volume particles (no mapping, section 3.3.4) are kept inside the closed
     mesh: the move is accepted iff the signed distance of y is negative
     (reading: the paper relies on repulsion alone; parity unpinned).
"""
from dataclasses import dataclass

import numpy as np

from . import force as F
from .geometry import barycentric, facet_frames, signed_distance_many

SURFACE, FEATURE, VOLUME = 2, 1, 3


def batch_facets(wl):
    """Facet frames of all geometries, indexed by global facet id."""
    parts = [facet_frames(g.mesh.vert, g.mesh.tri) for g in wl.geoms]
    return tuple(np.concatenate([p[k] for p in parts], 0) for k in range(4))


def batch_segments(wl):
    """Global segment table: start point, end point, length, unit tangent,
    first and one-past-last segment of the segment's line, closed flag."""
    p0, p1, lo, hi, closed = [], [], [], [], []
    for g in wl.geoms:
        L = g.mesh.lines
        p0.append(L.seg_p[:, 0])
        p1.append(L.seg_p[:, 1])
        for l in range(L.n_line):
            b, e = int(L.line_seg_begin[l]), int(L.line_seg_begin[l + 1])
            lo += [g.seg_begin + b] * (e - b)
            hi += [g.seg_begin + e] * (e - b)
            closed += [int(L.line_closed[l])] * (e - b)
    if not p0:
        z = np.zeros((0, 3))
        return z, z, np.zeros(0), z, np.zeros(0, int), np.zeros(0, int), np.zeros(0, int)
    p0 = np.concatenate(p0, 0)
    p1 = np.concatenate(p1, 0)
    ln = np.linalg.norm(p1 - p0, axis=1)
    t = (p1 - p0) / np.where(ln > 0, ln, 1.0)[:, None]
    return p0, p1, ln, t, np.array(lo, int), np.array(hi, int), np.array(closed, int)


@dataclass
class StepOut:
    a: np.ndarray          # [N, 3] acceleration (0 for non-moving)
    S: np.ndarray          # [N] force scale sum_j K(1-q/2)^3 |r_ij|
    nsrc: np.ndarray       # [N] number of sources
    amax: np.ndarray       # [G]
    tau: np.ndarray        # [G] dt^2
    dr: np.ndarray         # [N, 3] displacement after the tangential projection
    du: np.ndarray         # [N] arc-length increment of feature particles
    x_new: np.ndarray      # [N, 3] FP64 new position
    pos32: np.ndarray      # [N, 3] new position rounded to binary32
    owner: np.ndarray      # [N]
    feat_seg: np.ndarray   # [n_feat]
    feat_u: np.ndarray     # [n_feat]
    reverted: np.ndarray   # [N] bool
    margin: np.ndarray     # [N] bool: a decision within rounding of flipping


def time_step(wl, amax):
    """dt^2 = (h/16)/amax per geometry, 0 when nothing accelerates (parity unpinned)."""
    tau = np.zeros(len(wl.geoms))
    for g, geo in enumerate(wl.geoms):
        if amax[g] > 0:
            tau[g] = (float(geo.h) / 16.0) / amax[g]
    return tau


def displacement(wl, a, tau, owner, feat_seg, tag=None, gid=None):
    """Eq. 22-25 with the velocity reset: dr = tau a, restricted per class."""
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    mov = F.moving_mask(tag, wl.move_mask)
    dr = np.where(mov[:, None], tau[gid][:, None] * a, 0.0)
    du = np.zeros(len(dr))
    s = mov & (tag == SURFACE)
    if s.any():
        _, _, _, n = batch_facets(wl)
        nn = n[owner[s]]
        dr[s] = dr[s] - np.sum(dr[s] * nn, 1)[:, None] * nn
    f = mov & (tag == FEATURE)
    if f.any():
        _, _, _, t, _, _, _ = batch_segments(wl)
        tt = t[feat_seg[owner[f]]]
        du[f] = np.sum(dr[f] * tt, 1)
        dr[f] = du[f][:, None] * tt
    return dr, du


def project_surface(wl, y, g, lam_margin=1e-7, d_margin=1e-9):
    """Section 3.3.3 reprojection of points y [P, 3] of geometry g, brute force
    over all its facets. Returns (accepted, foot point, global facet, margin)."""
    geo = wl.geoms[g]
    A, B, C, n = facet_frames(geo.mesh.vert, geo.mesh.tri)
    ids = np.arange(len(A))
    ok = np.zeros(len(y), bool)
    foot = y.copy()
    own = np.full(len(y), -1, np.int64)
    margin = np.zeros(len(y), bool)
    filt = csg_filter(geo)
    for s in range(0, len(y), 256):
        o, f, w, m = project_onto_facets(y[s:s + 256], A, B, C, n, ids, float(geo.proj_radius),
                                         lam_margin, d_margin, filt)
        ok[s:s + 256], foot[s:s + 256], margin[s:s + 256] = o, f, m
        own[s:s + 256] = np.where(o, w + geo.tri_begin, -1)
    return ok, foot, own, margin


def csg_filter(geo):
    """For a Boolean assembly: the test that a foot point on a facet lies on the
    assembly's boundary (csg.on_boundary); None for a single mesh."""
    if getattr(geo, "csg", None) is None:
        return None
    from . import csg
    return lambda p, facets: csg.on_boundary(p, facets, geo)


def project_onto_facets(y, A, B, C, n, ids, R, lam_margin=1e-7, d_margin=1e-9, filt=None):
    """The section 3.3.3 decision for points y [P, 3] over the facets (A, B, C,
    n) whose local indices `ids` are ascending: plane distance d, foot point
    p = y - d n, accepted iff every barycentric coordinate of p is >= 0 and
    |d| <= R (and, for a Boolean assembly, `filt` places p on its boundary);
    the accepted facet with the smallest |d| wins, ties to the lowest index.
    Returns (accepted, foot, winning index from ids, margin)."""
    q = y[:, None, :]
    d = np.sum((q - A[None]) * n[None], -1)                     # [P, T] signed plane distance
    p = q - d[..., None] * n[None]
    la, lb, lc = barycentric(p, A[None], B[None], C[None])
    lmin = np.minimum(np.minimum(la, lb), lc)
    ad = np.abs(d)
    acc = (lmin >= 0) & (ad <= R)
    csg_margin = np.zeros(len(y), bool)
    if filt is not None and acc.any():
        r, c = np.nonzero(acc)
        ok, near = filt(p[r, c], np.asarray(ids)[c])
        acc[r[~ok], c[~ok]] = False
        csg_margin[r[near]] = True
    key = np.where(acc, ad, np.inf)
    best = np.argmin(key, axis=1)                                # first index among equal minima
    has = np.isfinite(key[np.arange(len(best)), best])
    foot = y.copy()
    rows = np.nonzero(has)[0]
    foot[rows] = p[rows, best[rows]]
    # decisions that rounding could flip: the winner's foot point on its
    # facet boundary or its |d| at the radius, another facet on the edge of
    # acceptance that would beat the winner, or two accepted facets within
    # d_margin of each other
    bd = np.where(has, key[np.arange(len(best)), best], np.inf)
    edge = (np.abs(lmin) <= lam_margin) & (ad <= np.minimum(bd, R)[:, None] + d_margin)
    near_R = has & (np.abs(bd - R) <= d_margin)
    srt = np.sort(key, axis=1)
    with np.errstate(invalid="ignore"):                          # inf - inf where nothing is accepted
        tie = (np.isfinite(srt[:, 1]) & (srt[:, 1] - srt[:, 0] <= d_margin)) if key.shape[1] > 1 \
            else np.zeros(len(best), bool)
    return has, foot, np.asarray(ids)[best], edge.any(1) | near_R | tie | csg_margin


def advance_feature(seg, u, du, segs, margin_tol=1e-9):
    """Move a feature particle by arc length du along its polyline (parity
    unpinned reading). Returns (accepted, segment, u, margin)."""
    p0, p1, ln, t, lo, hi, closed = segs
    s = int(seg)
    v = float(u) + float(du)
    margin = False
    for _ in range(hi[s] - lo[s] + 2):
        if v < 0.0:
            margin |= v > -margin_tol
            if s > lo[s]:
                s -= 1
                v += ln[s]
            elif closed[s]:
                s = hi[s] - 1
                v += ln[s]
            else:
                return False, int(seg), float(u), margin
        elif v > ln[s]:
            margin |= v - ln[s] < margin_tol
            if s < hi[s] - 1:
                v -= ln[s]
                s += 1
            elif closed[s]:
                v -= ln[s]
                s = lo[s]
            else:
                return False, int(seg), float(u), margin
        else:
            margin |= (v < margin_tol) or (ln[s] - v < margin_tol)
            return True, s, v, margin
    raise RuntimeError("feature walk did not terminate")


def relax_step(wl, pos32=None, owner=None, feat_seg=None, feat_u=None, tag=None, gid=None,
               sd_margin=1e-6, accel_override=None) -> StepOut:
    """Algorithm 1, one iteration, for all particles of the workload.
    accel_override = (a, S, counts, amax) replaces the force and its maximum
    (the multi-resolution step of multires.py)."""
    pos32 = wl.pos if pos32 is None else np.asarray(pos32, np.float32)
    owner = wl.owner if owner is None else np.asarray(owner)
    feat_seg = wl.feat_seg if feat_seg is None else np.asarray(feat_seg)
    feat_u = wl.feat_u if feat_u is None else np.asarray(feat_u, np.float64)
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    if accel_override is None:
        a, S, cnt = F.accel(wl, None, pos32, tag, gid)
        amax = F.amax_per_geometry(wl, a, tag, gid)
    else:
        a, S, cnt, amax = accel_override
    tau = time_step(wl, amax)
    dr, du = displacement(wl, a, tau, owner, feat_seg, tag, gid)
    mov = F.moving_mask(tag, wl.move_mask)
    x = pos32.astype(np.float64)
    x_new = x.copy()
    owner_new = np.array(owner, copy=True)
    fs_new = np.array(feat_seg, copy=True)
    fu_new = np.array(feat_u, copy=True)
    reverted = np.zeros(len(x), bool)
    margin = np.zeros(len(x), bool)
    for g, geo in enumerate(wl.geoms):
        s = np.nonzero(mov & (gid == g) & (tag == SURFACE))[0]
        if len(s):
            y = x[s] + dr[s]
            ok, foot, own, mg = project_surface(wl, y, g)
            x_new[s[ok]] = foot[ok]
            owner_new[s[ok]] = own[ok]
            reverted[s[~ok]] = True
            margin[s] = mg
        v = np.nonzero(mov & (gid == g) & (tag == VOLUME))[0]
        if len(v):
            y = x[v] + dr[v]
            if getattr(geo, "csg", None) is not None:
                from . import csg
                sd = csg.assembly_sd(y, geo)
            else:
                sd = signed_distance_many(y, geo.mesh.vert, geo.mesh.tri)
            ok = sd < 0
            x_new[v[ok]] = y[ok]
            reverted[v[~ok]] = True
            margin[v] = np.abs(sd) <= sd_margin
    f = np.nonzero(mov & (tag == FEATURE))[0]
    if len(f):
        segs = batch_segments(wl)
        p0, p1, ln = segs[0], segs[1], segs[2]
        for i in f:
            slot = owner[i]
            ok, sg, u, mg = advance_feature(feat_seg[slot], feat_u[slot], du[i], segs)
            margin[i] = mg
            if ok:
                fs_new[slot], fu_new[slot] = sg, u
                x_new[i] = p0[sg] + (u / ln[sg]) * (p1[sg] - p0[sg])
            else:
                reverted[i] = True
    pos_new32 = x_new.astype(np.float32)
    pos_new32[~mov] = pos32[~mov]
    pos_new32[reverted] = pos32[reverted]
    return StepOut(a=a, S=S, nsrc=cnt, amax=amax, tau=tau, dr=dr, du=du, x_new=x_new,
                   pos32=pos_new32, owner=owner_new, feat_seg=fs_new, feat_u=fu_new,
                   reverted=reverted, margin=margin)
