"""Full-size mode of the step oracle (TEST INFRASTRUCTURE ONLY, like the rest
of this package).

The brute-force oracle tests every receiver against every particle and every
point against every facet, which does not finish at millions of particles.
This module computes the same iteration (step.py: Eq. 15-17 forces, the time
step, Eq. 22-25 displacement, the section 3.3.3 projection, the feature walk,
the volume rule) with the searches narrowed to candidate sets that provably
contain everything the definition can accept, and with the per-pair and
per-facet arithmetic of force.py and step.py:

  neighbours   the binary32 predicate of neighbors.py can only hold for pairs
               whose FP64 distance is below rc (1 + 8 u), u = 2^-24 (each of
               the eight binary32 operations of the predicate has relative
               error at most u and rc2 = fl32(fl32(2h)^2) <= (2h)^2 (1 + u)^2).
               Candidates: the particles of the 27 cells around a receiver in
               a grid of cell edge rc (1 + 1e-6) >= that bound, then the
               binary32 predicate itself.
  projection   an accepted foot point lies on its facet within |d| <= R of y,
               so y lies in the facet's bounding box widened by R; the margin
               tests look at facets whose foot lies within 1e-7 (barycentric)
               of the facet and whose |d| is within R + 1e-9. Candidates: the
               facets registered in y's cell of a grid, each facet in every
               cell its bounding box widened by R (1 + 1e-3) + 1e-6 (1 + its
               extent) touches; the decision is then step.project_onto_facets
               over those facets in ascending order (the same argmin, ties to
               the lowest facet).
  volume rule  sd(y) < 0 with sd = sigma min dist (step.py). sigma from the
               winding number, here computed as the signed count of facets a
               vertical ray from y crosses (+1 where the outward normal points
               up, -1 where down): for a closed mesh and a ray that meets no
               edge, the solid-angle sum of geometry.winding_number equals that
               count. Rays within 1e-12 (barycentric) of an edge, or points
               within 1e-12 of a facet plane at the crossing, fall back to the
               solid-angle sum. The distance, needed only to flag |sd| <=
               sd_margin and sd = 0, from the facets registered in y's cell.

Pinned against the brute-force oracle on small cases (tests/test_oracle_local.py).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import force as F
from .geometry import facet_frames, winding_number, unsigned_distance_many
from .kernel import force_coef
from .neighbors import pair_d2_xyz, rc2_f32
from . import csg
from .step import (FEATURE, SURFACE, VOLUME, StepOut, advance_feature, batch_segments, csg_filter, displacement,
                   project_onto_facets, time_step)

RANK = F.RANK


# ---------------------------------------------------------------------------- neighbours

def _cells(p64, edge):
    lo = p64.min(0) - 2 * edge
    t = (p64 - lo) / edge
    c = np.floor(t).astype(np.int64)
    dims = c.max(0) + 3
    key = (c[:, 2] * dims[1] + c[:, 1]) * dims[0] + c[:, 0]
    order = np.argsort(key, kind="stable")
    start = np.zeros(int(np.prod(dims)) + 1, np.int64)
    np.add.at(start, key + 1, 1)
    return c, dims, order, np.cumsum(start), t - c


_OFFS = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)], np.int64)


def candidate_pairs(pos32, receivers, rc, chunk=1 << 14, grid=None):
    """Yield (r, j) index arrays: for each receiver index r (into pos32) the
    particles j of the 27 cells around it, in a grid of cell edge rc (1 + 1e-6),
    whose box comes within that edge of the receiver (a superset of every pair
    the binary32 predicate can accept); the caller applies the predicate."""
    reach = rc * (1.0 + 1e-6)
    c, dims, order, start, frac = grid or _cells(pos32.astype(np.float64), reach)
    for s in range(0, len(receivers), chunk):
        r = receivers[s:s + chunk]
        rs, js = [], []
        cr, fr = c[r], frac[r]
        for o in _OFFS:
            # distance in cell units from the receiver to the box of cell c + o, per axis
            g = np.where(o > 0, o - fr, np.where(o < 0, fr + (-o - 1), 0.0))
            near = np.nonzero(np.sum(g * g, axis=1) <= 1.0)[0]          # (gap * edge)^2 <= reach^2
            if len(near) == 0:
                continue
            cc = cr[near] + o
            key = (cc[:, 2] * dims[1] + cc[:, 1]) * dims[0] + cc[:, 0]   # in range: the grid has a margin
            b, e = start[key], start[key + 1]
            cnt = e - b
            tot = int(cnt.sum())
            if tot == 0:
                continue
            first = np.cumsum(cnt) - cnt
            j = order[np.repeat(b, cnt) + (np.arange(tot) - np.repeat(first, cnt))]
            rs.append(np.repeat(r[near], cnt))
            js.append(j)
        if rs:
            yield np.concatenate(rs), np.concatenate(js)


def accel(wl, receivers=None, pos32=None, tag=None, gid=None, threads=None):
    """force.accel over candidate pairs: (a [R, 3], S [R], source count [R]).
    The receivers are processed in chunks by `threads` threads (default: the
    CPUs this process may use, at most 16); every receiver's sums come from
    one chunk, so the result does not depend on the thread count."""
    pos32 = wl.pos if pos32 is None else pos32
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    receivers = np.arange(len(pos32)) if receivers is None else np.asarray(receivers)
    mov = F.moving_mask(tag, wl.move_mask)
    a = np.zeros((len(receivers), 3))
    S = np.zeros(len(receivers))
    cnt = np.zeros(len(receivers), np.int64)
    slot = np.full(len(pos32), -1, np.int64)
    slot[receivers] = np.arange(len(receivers))
    x64 = pos32.astype(np.float64)
    for g, geo in enumerate(wl.geoms):
        members = np.nonzero(gid == g)[0]
        sel = receivers[(gid[receivers] == g) & mov[receivers]]
        if len(sel) == 0:
            continue
        h = float(geo.h)
        K = force_coef(h)
        rc2 = rc2_f32(geo.h)
        rc = float(np.float32(2.0) * np.float32(h))
        loc = np.full(len(pos32), -1, np.int64)
        loc[members] = np.arange(len(members))
        pm32 = pos32[members]
        px, py, pz = (np.ascontiguousarray(pm32[:, q]) for q in range(3))
        p64 = [x64[members, q].copy() for q in range(3)]
        rank_m = RANK[tag[members]]
        grid = _cells(pm32.astype(np.float64), rc * (1.0 + 1e-6))
        # receivers in cell order (the candidate gathers stay local), in chunks
        rl = loc[sel]
        rl = rl[np.argsort((grid[0][rl, 2] * grid[1][1] + grid[0][rl, 1]) * grid[1][0] + grid[0][rl, 0],
                           kind="stable")]
        chunks = [rl[q:q + (1 << 14)] for q in range(0, len(rl), 1 << 14)]

        def work(chunk):
            out = []
            for ri, jj in candidate_pairs(pm32, chunk, rc, grid=grid):
                out.append(_pair_sums(ri, jj))
            return out

        def _pair_sums(ri, jj):
            keep = (ri != jj) & (pair_d2_xyz(px[ri], py[ri], pz[ri], px[jj], py[jj], pz[jj]) < rc2)
            keep &= rank_m[jj] <= rank_m[ri]
            ri, jj = ri[keep], jj[keep]
            i = members[ri]
            d = np.stack([p64[q][ri] - p64[q][jj] for q in range(3)], axis=1)   # FP64 r_ij
            dist = np.sqrt(np.einsum("pk,pk->p", d, d))
            t = np.clip(1.0 - 0.5 * dist / h, 0.0, None)
            w = K * t ** 3
            k = slot[i]
            u, inv = np.unique(k, return_inverse=True)
            sums = [np.bincount(inv, weights=w * d[:, q], minlength=len(u)) for q in range(3)]
            return u, sums, np.bincount(inv, weights=w * dist, minlength=len(u)), \
                np.bincount(inv, minlength=len(u))

        nt = threads or min(16, len(os.sched_getaffinity(0)))
        with ThreadPoolExecutor(max_workers=max(1, nt)) as ex:
            for res in ex.map(work, chunks):
                for u, sums, s_, c_ in res:          # each receiver's pairs come from one chunk
                    for q in range(3):
                        a[u, q] += sums[q]
                    S[u] += s_
                    cnt[u] += c_
    return a, S, cnt


# ---------------------------------------------------------------------------- facet candidates

class FacetGrid:
    """Facets of one mesh registered in the cells of a uniform grid that their
    bounding box, widened by pad + 1e-6 (1 + extent), touches."""

    def __init__(self, vert, tri, pad, edge=None):
        A, B, C, n = facet_frames(vert, tri)
        self.A, self.B, self.C, self.n = A, B, C, n
        lo3 = np.minimum(np.minimum(A, B), C)
        hi3 = np.maximum(np.maximum(A, B), C)
        ext = np.max(hi3 - lo3, axis=1)
        w = pad + 1e-6 * (1.0 + ext)
        lo3 = lo3 - w[:, None]
        hi3 = hi3 + w[:, None]
        if edge is None:
            edge = max(2.0 * pad, float(np.median(ext)), 1e-9)
        self.edge = edge
        self.lo = lo3.min(0)
        self.dims = np.floor((hi3.max(0) - self.lo) / edge).astype(np.int64) + 1
        c0 = np.floor((lo3 - self.lo) / edge).astype(np.int64)
        c1 = np.floor((hi3 - self.lo) / edge).astype(np.int64)
        span = c1 - c0 + 1
        cnt = np.prod(span, axis=1)
        fid = np.repeat(np.arange(len(tri)), cnt)
        k = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        sx, sy = np.repeat(span[:, 0], cnt), np.repeat(span[:, 1], cnt)
        cx = np.repeat(c0[:, 0], cnt) + k % sx
        cy = np.repeat(c0[:, 1], cnt) + (k // sx) % sy
        cz = np.repeat(c0[:, 2], cnt) + k // (sx * sy)
        key = (cz * self.dims[1] + cy) * self.dims[0] + cx
        o = np.lexsort((fid, key))                      # by cell, facets ascending inside a cell
        self.key = key[o]
        self.fid = fid[o]

    def cell_of(self, p):
        c = np.floor((p - self.lo) / self.edge).astype(np.int64)
        inside = np.all((c >= 0) & (c < self.dims), axis=1)
        c = np.clip(c, 0, self.dims - 1)
        return np.where(inside, (c[:, 2] * self.dims[1] + c[:, 1]) * self.dims[0] + c[:, 0], -1)

    def groups(self, p):
        """Yield (point indices, ascending facet ids) per occupied cell; points
        outside the grid or in a cell without facets are yielded with an empty
        facet list."""
        cell = self.cell_of(p)
        o = np.argsort(cell, kind="stable")
        cs = cell[o]
        bnd = np.nonzero(np.diff(cs))[0] + 1
        for grp in np.split(o, bnd):
            if len(grp) == 0:
                continue
            k = cell[grp[0]]
            if k < 0:
                yield grp, np.zeros(0, np.int64)
                continue
            a, b = np.searchsorted(self.key, k), np.searchsorted(self.key, k, side="right")
            yield grp, self.fid[a:b]


def project_surface(wl, y, g, lam_margin=1e-7, d_margin=1e-9, grid=None):
    """step.project_surface over the candidate facets of each point."""
    geo = wl.geoms[g]
    R = float(geo.proj_radius)
    grid = grid or FacetGrid(geo.mesh.vert, geo.mesh.tri, R * (1.0 + 1e-3) + 1e-6)
    filt = csg_filter(geo)
    ok = np.zeros(len(y), bool)
    foot = y.copy()
    own = np.full(len(y), -1, np.int64)
    margin = np.zeros(len(y), bool)
    for pts, fac in grid.groups(y):
        if len(fac) == 0:
            continue
        o, f, w, m = project_onto_facets(y[pts], grid.A[fac], grid.B[fac], grid.C[fac], grid.n[fac], fac, R,
                                         lam_margin, d_margin, filt)
        ok[pts], foot[pts], margin[pts] = o, f, m
        own[pts] = np.where(o, w + geo.tri_begin, -1)
    return ok, foot, own, margin


# ---------------------------------------------------------------------------- inside / outside

def ray_winding(p, vert, tri, eps=1e-12):
    """Winding number of a closed outward mesh at points p [P, 3] as the signed
    number of facets crossed by the ray from p towards +z (+1 for an outward
    normal with a positive z component, -1 for a negative one). Points whose
    ray passes within eps (barycentric) of a facet edge, or that lie within
    eps of the crossing, get the solid-angle winding number instead."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    A = vert[tri[:, 0]]
    B = vert[tri[:, 1]]
    C = vert[tri[:, 2]]
    area2 = (B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (B[:, 1] - A[:, 1]) * (C[:, 0] - A[:, 0])
    use = np.nonzero(area2 != 0.0)[0]                   # vertical facets are never crossed
    lo = np.minimum(np.minimum(A[use, :2], B[use, :2]), C[use, :2])
    hi = np.maximum(np.maximum(A[use, :2], B[use, :2]), C[use, :2])
    ext = float(np.median(np.max(hi - lo, axis=1))) if len(use) else 1.0
    edge = max(ext, 1e-9)
    glo = lo.min(0) - edge if len(use) else np.zeros(2)
    dims = (np.floor(((hi.max(0) if len(use) else np.ones(2)) - glo) / edge).astype(np.int64) + 2)
    c0 = np.floor((lo - glo) / edge).astype(np.int64)
    c1 = np.floor((hi - glo) / edge).astype(np.int64)
    span = c1 - c0 + 1
    cnt = span[:, 0] * span[:, 1]
    fid = np.repeat(use, cnt)
    k = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    sx = np.repeat(span[:, 0], cnt)
    key = (np.repeat(c0[:, 1], cnt) + k // sx) * dims[0] + np.repeat(c0[:, 0], cnt) + k % sx
    o = np.lexsort((fid, key))
    key, fid = key[o], fid[o]
    wn = np.zeros(len(p))
    fallback = np.zeros(len(p), bool)
    cp = np.floor((p[:, :2] - glo) / edge).astype(np.int64)
    inside = np.all((cp >= 0) & (cp < dims), axis=1)
    ck = np.where(inside, cp[:, 1] * dims[0] + cp[:, 0], -1)
    order = np.argsort(ck, kind="stable")
    bnd = np.nonzero(np.diff(ck[order]))[0] + 1
    for grp in np.split(order, bnd):
        kk = ck[grp[0]]
        if kk < 0:
            continue
        a, b = np.searchsorted(key, kk), np.searchsorted(key, kk, side="right")
        f = fid[a:b]
        if len(f) == 0:
            continue
        q = p[grp][:, None, :]
        ar = area2[f][None]
        lb = ((q[..., 0] - A[f, 0]) * (C[f, 1] - A[f, 1]) - (q[..., 1] - A[f, 1]) * (C[f, 0] - A[f, 0])) / ar
        lc = ((B[f, 0] - A[f, 0]) * (q[..., 1] - A[f, 1]) - (B[f, 1] - A[f, 1]) * (q[..., 0] - A[f, 0])) / ar
        la = 1.0 - lb - lc
        z = la * A[f, 2] + lb * B[f, 2] + lc * C[f, 2]
        lmin = np.minimum(np.minimum(la, lb), lc)
        hit = (lmin > eps) & (z > q[..., 2] + eps)
        wn[grp] = np.sum(np.where(hit, np.sign(ar), 0.0), axis=1)
        near = (np.abs(lmin) <= eps) & (z > q[..., 2] - eps)      # ray through an edge or vertex
        near |= (lmin > -eps) & (np.abs(z - q[..., 2]) <= eps)    # point at the crossing
        fallback[grp] = near.any(1)
    if fallback.any():
        wn[fallback] = winding_number(p[fallback], vert, tri)
    return wn


def volume_rule(y, mesh, sd_margin=1e-6, grid=None):
    """step.py's volume rule: (accepted = sd(y) < 0, margin = |sd(y)| <= sd_margin)."""
    wn = ray_winding(y, mesh.vert, mesh.tri)
    grid = grid or FacetGrid(mesh.vert, mesh.tri, sd_margin)
    d = np.full(len(y), np.inf)                         # inf: farther than the grid's pad from every facet
    for pts, fac in grid.groups(y):
        if len(fac):
            d[pts] = unsigned_distance_many(y[pts], mesh.vert, mesh.tri[fac])
    sigma = np.where(wn > 0.5, -1.0, 1.0)
    sd = sigma * d
    return sd < 0, np.abs(sd) <= sd_margin


# ---------------------------------------------------------------------------- one iteration

def relax_step(wl, pos32=None, owner=None, feat_seg=None, feat_u=None, tag=None, gid=None, sd_margin=1e-6,
               a=None, sample=None):
    """step.relax_step with the candidate searches above. `a` may pass the
    accelerations of all particles already computed by accel() (the same
    positions). sample (boolean mask, optional): the forces, amax and
    displacements are still those of every particle, but only the sampled
    moving particles are projected; the others keep their position and are
    neither reverted nor margin cases."""
    pos32 = wl.pos if pos32 is None else np.asarray(pos32, np.float32)
    owner = wl.owner if owner is None else np.asarray(owner)
    feat_seg = wl.feat_seg if feat_seg is None else np.asarray(feat_seg)
    feat_u = wl.feat_u if feat_u is None else np.asarray(feat_u, np.float64)
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    mov = F.moving_mask(tag, wl.move_mask)
    proj = mov if sample is None else (mov & np.asarray(sample, bool))
    if a is None:
        a, S, cnt = accel(wl, None, pos32, tag, gid)
    else:
        S = cnt = None
    amax = F.amax_per_geometry(wl, a, tag, gid)
    tau = time_step(wl, amax)
    dr, du = displacement(wl, a, tau, owner, feat_seg, tag, gid)
    x = pos32.astype(np.float64)
    x_new = x.copy()
    owner_new = np.array(owner, copy=True)
    fs_new = np.array(feat_seg, copy=True)
    fu_new = np.array(feat_u, copy=True)
    reverted = np.zeros(len(x), bool)
    margin = np.zeros(len(x), bool)
    for g, geo in enumerate(wl.geoms):
        s = np.nonzero(proj & (gid == g) & (tag == SURFACE))[0]
        if len(s):
            y = x[s] + dr[s]
            ok, foot, own, mg = project_surface(wl, y, g)
            x_new[s[ok]] = foot[ok]
            owner_new[s[ok]] = own[ok]
            reverted[s[~ok]] = True
            margin[s] = mg
        v = np.nonzero(proj & (gid == g) & (tag == VOLUME))[0]
        if len(v):
            y = x[v] + dr[v]
            if getattr(geo, "csg", None) is not None:   # parts have few facets: the brute-force rule
                sd = csg.assembly_sd(y, geo)
                ok, mg = sd < 0, np.abs(sd) <= sd_margin
            else:
                ok, mg = volume_rule(y, geo.mesh, sd_margin)
            x_new[v[ok]] = y[ok]
            reverted[v[~ok]] = True
            margin[v] = mg
    f = np.nonzero(proj & (tag == FEATURE))[0]
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
    pos_new32[~proj] = pos32[~proj]
    pos_new32[reverted] = pos32[reverted]
    return StepOut(a=a, S=S, nsrc=cnt, amax=amax, tau=tau, dr=dr, du=du, x_new=x_new,
                   pos32=pos_new32, owner=owner_new, feat_seg=fs_new, feat_u=fu_new,
                   reverted=reverted, margin=margin)
