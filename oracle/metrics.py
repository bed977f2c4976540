"""Convergence and quality measures of a particle distribution.

The paper judges uniformity visually and gives no formula (parity unpinned
readings):
  * force residual  R(x) = sqrt( mean over moving i of |P_i a_i|^2 ), with
    P_i = I - n n^T for a surface particle (n: owner facet normal), t t^T for a
    feature particle (t: owner segment tangent), I for a volume particle.
  * uniformity loss  L(x) = mean over moving i of (rho_i / rho_0 - 1)^2, with
    the kernel density rho_i = W(0) + sum_{j: pred(i, j)} W(r_ij) over all
    classes (the kernel sum of Eq. 7) and rho_0 the same sum over an infinite
    cubic lattice of spacing dx.
"""
import numpy as np

from . import force as F
from .kernel import W
from .neighbors import pair_d2, rc2_f32
from .step import batch_facets, batch_segments

SURFACE, FEATURE = 2, 1


def projected_accel(wl, a, owner, feat_seg, tag=None):
    tag = wl.tag if tag is None else tag
    pa = np.array(a, np.float64, copy=True)
    s = tag == SURFACE
    if s.any():
        _, _, _, n = batch_facets(wl)
        nn = n[owner[s]]
        pa[s] -= np.sum(pa[s] * nn, 1)[:, None] * nn
    f = tag == FEATURE
    if f.any():
        t = batch_segments(wl)[3]
        tt = t[feat_seg[owner[f]]]
        pa[f] = np.sum(pa[f] * tt, 1)[:, None] * tt
    return pa


def residual(wl, a, owner, feat_seg, tag=None):
    tag = wl.tag if tag is None else tag
    mov = F.moving_mask(tag, wl.move_mask)
    pa = projected_accel(wl, a, owner, feat_seg, tag)
    return float(np.sqrt(np.mean(np.sum(pa[mov] ** 2, 1)))) if mov.any() else 0.0


def lattice_density(dx: float, h: float) -> float:
    """rho_0: W(0) + sum of W over all non-zero points of the cubic lattice dx Z^3 within 2h."""
    m = int(np.ceil(2.0 * h / dx)) + 1
    r = np.arange(-m, m + 1) * dx
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    return float(np.sum(W(np.linalg.norm(g, axis=1), h)))


def densities(wl, pos32=None, tag=None, gid=None):
    pos32 = wl.pos if pos32 is None else pos32
    gid = wl.gid if gid is None else gid
    rho = np.zeros(len(pos32))
    x = pos32.astype(np.float64)
    for g, geo in enumerate(wl.geoms):
        members = np.nonzero(gid == g)[0]
        rc2 = rc2_f32(geo.h)
        h = float(geo.h)
        step = max(1, (1 << 24) // max(len(members), 1))
        for s in range(0, len(members), step):
            r = members[s:s + step]
            hit = pair_d2(pos32[r][:, None, :], pos32[members][None, :, :]) < rc2
            hit &= members[None, :] != r[:, None]
            b, m = np.nonzero(hit)
            d = np.linalg.norm(x[r[b]] - x[members[m]], axis=1)
            rho[r] = W(0.0, h) + np.bincount(b, weights=W(d, h), minlength=len(r))
    return rho


def uniformity_loss(wl, pos32=None, tag=None, gid=None):
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    rho = densities(wl, pos32, tag, gid)
    mov = F.moving_mask(tag, wl.move_mask)
    rho0 = np.array([lattice_density(g.dx, float(g.h)) for g in wl.geoms])[gid]
    return float(np.mean((rho[mov] / rho0[mov] - 1.0) ** 2)) if mov.any() else 0.0
