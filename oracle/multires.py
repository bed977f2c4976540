"""Multi-resolution relaxation (the paper's stated future work, Conclusions;
the pair smoothing length h_ij = (h_i + h_j) / 2 of Eq. 6).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Reading (the paper gives no multi-resolution method; parity unpinned as a
reading, pinned below by its reductions and invariants):

  level        every particle has a level l_i in {0, 1, 2, 3} and the
               smoothing length h_i = h 2^-l_i, h the geometry's (coarsest)
               smoothing length
  pair         h_ij = (h_i + h_j) / 2; j is a neighbour of i iff the binary32
               test |r_ij|^2 < fl32(fl32(h_i + h_j)^2) (the support 2 h_ij,
               same summation order as the single-resolution predicate)
  force        a_i = sum_{j in src(i)} K(h_ij) (1 - r_ij / (2 h_ij))^3 r_ij with
               K(h) = 5 alpha(h) / h^2 (Eq. 15-17 at the pair's length), over
               the rank rule of section 2.2
  time step    each moving particle moves at most h_i / 16: dt^2 =
               (h / 16) / max_i (|a_i| 2^l_i) per geometry (with all levels 0
               the single-resolution rule)
  the rest     projection, reverts and feature walks as in step.py

With every level 0 it is the single-resolution step (pinned).
"""
import numpy as np

from . import force as F
from . import step as S
from .kernel import force_coef
from .neighbors import pair_d2

MAX_LEVEL = 3


def h_of(geo, level):
    """h_i = h 2^-l (binary32 h scaled by a power of two: exact)."""
    return np.float32(geo.h) * np.exp2(-np.asarray(level, np.float64)).astype(np.float32)


def accel(wl, level, receivers=None, pos32=None, tag=None, gid=None, chunk=256):
    """a [R, 3], S [R] = sum_j K_ij (1 - r/2h_ij)^3 |r_ij| and source counts
    for the receivers (default all), with per-particle levels."""
    pos32 = wl.pos if pos32 is None else pos32
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    level = np.asarray(level, np.int64)
    receivers = np.arange(len(pos32)) if receivers is None else np.asarray(receivers)
    mov = F.moving_mask(tag, wl.move_mask)
    a = np.zeros((len(receivers), 3))
    Ssum = np.zeros(len(receivers))
    cnt = np.zeros(len(receivers), np.int64)
    x64 = pos32.astype(np.float64)
    for g, geo in enumerate(wl.geoms):
        members = np.nonzero(gid == g)[0]
        pm32 = pos32[members]
        rank_m = F.RANK[tag[members]]
        hm = h_of(geo, level[members])                         # binary32 [M]
        sel = np.nonzero((gid[receivers] == g) & mov[receivers])[0]
        step = max(1, min(chunk, (1 << 24) // max(len(members), 1)))
        for s in range(0, len(sel), step):
            rows = sel[s:s + step]
            r = receivers[rows]
            hr = h_of(geo, level[r])
            hs = (hr[:, None] + hm[None, :]).astype(np.float32)  # fl32(h_i + h_j)
            rc2 = (hs * hs).astype(np.float32)
            hit = pair_d2(pos32[r][:, None, :], pm32[None, :, :]) < rc2
            hit &= members[None, :] != r[:, None]
            hit &= rank_m[None, :] <= F.RANK[tag[r]][:, None]
            b, m = np.nonzero(hit)
            hij = 0.5 * (hr[b].astype(np.float64) + hm[m].astype(np.float64))
            d = x64[r[b]] - x64[members[m]]
            dist = np.sqrt(np.einsum("pk,pk->p", d, d))
            t = np.clip(1.0 - 0.5 * dist / hij, 0.0, None)
            K = np.array([force_coef(float(v)) for v in hij]) if len(hij) else np.zeros(0)
            w = K * t ** 3
            for k in range(3):
                a[rows, k] = np.bincount(b, weights=w * d[:, k], minlength=len(rows))
            Ssum[rows] = np.bincount(b, weights=w * dist, minlength=len(rows))
            cnt[rows] = np.bincount(b, minlength=len(rows))
    return a, Ssum, cnt


def amax_per_geometry(wl, a, level, tag=None, gid=None):
    """max over the geometry's moving particles of |a_i| 2^l_i."""
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    mov = F.moving_mask(tag, wl.move_mask)
    scaled = np.linalg.norm(a, axis=1) * np.exp2(np.asarray(level, np.float64))
    out = np.zeros(len(wl.geoms))
    for g in range(len(wl.geoms)):
        sel = mov & (gid == g)
        if sel.any():
            out[g] = scaled[sel].max()
    return out


def relax_step(wl, level, pos32=None):
    """One iteration with levels: the multi-resolution force and time step,
    then the displacement, projection, reverts and feature walks of
    step.relax_step (whose force and amax are replaced)."""
    pos32 = wl.pos if pos32 is None else np.asarray(pos32, np.float32)
    a, Ssum, cnt = accel(wl, level, None, pos32)
    amax = amax_per_geometry(wl, a, level)
    return S.relax_step(wl, pos32=pos32, accel_override=(a, Ssum, cnt, amax))
