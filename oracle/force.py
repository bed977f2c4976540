"""Relaxation acceleration, Eq. 15 (section 3.3.1), brute force in FP64.

    a_i = sum_{j in src(i)} K (1 - q_ij/2)^3 (x_i - x_j),   q_ij = |x_i - x_j| / h

which is -sum_j dW/dr(r_ij) e_ij with the Wendland C2 kernel and prefactor 1
(see kernel.py). Neighbours are the pairs passing the binary32 predicate of
neighbors.py; the distance inside the force is exact FP64 of the binary32
coordinates, with the factor (1 - q/2) clipped at 0 (W is 0 outside q <= 2).

Interaction rule between particle classes (section 2.2; section 3.3.3 and
3.3.4): every class is acted on by its own class and by the classes that bound
it, never by the classes it bounds. With ranks
    singular 0, feature 1, surface 2, volume 3, fixed volume 3,
source j acts on receiver i iff rank(j) <= rank(i). Only moving receivers
(tag bit set in move_mask, singular and fixed never) get an acceleration; the
others get 0.
"""
import numpy as np

from .kernel import force_coef
from .neighbors import pair_d2, rc2_f32

RANK = np.array([0, 1, 2, 3, 3], np.int64)


def moving_mask(tag: np.ndarray, move_mask: int) -> np.ndarray:
    tag = np.asarray(tag, np.int64)
    return (((move_mask >> tag) & 1) == 1) & (tag >= 1) & (tag <= 3)


def accel(wl, receivers=None, pos32=None, tag=None, gid=None, chunk=256, pos64=None):
    """Acceleration a [R, 3], scale S [R] = sum_j K (1-q/2)^3 |r_ij| and source
    count [R] for the receivers (default: all particles).

    The neighbour sets come from the binary32 positions; the pair vectors from
    `pos64` when given (to differentiate at fixed neighbour sets), else from the
    binary32 positions converted exactly to FP64."""
    pos32 = wl.pos if pos32 is None else pos32
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    receivers = np.arange(len(pos32)) if receivers is None else np.asarray(receivers)
    mov = moving_mask(tag, wl.move_mask)
    a = np.zeros((len(receivers), 3))
    S = np.zeros(len(receivers))
    cnt = np.zeros(len(receivers), np.int64)
    x64 = pos32.astype(np.float64) if pos64 is None else np.asarray(pos64, np.float64)
    for g, geo in enumerate(wl.geoms):
        members = np.nonzero(gid == g)[0]
        pm32 = pos32[members]
        pm64 = x64[members]
        rank_m = RANK[tag[members]]
        h = float(geo.h)
        K = force_coef(h)
        rc2 = rc2_f32(geo.h)
        sel = np.nonzero((gid[receivers] == g) & mov[receivers])[0]
        step = max(1, min(chunk, (1 << 24) // max(len(members), 1)))
        for s in range(0, len(sel), step):
            rows = sel[s:s + step]
            r = receivers[rows]
            hit = pair_d2(pos32[r][:, None, :], pm32[None, :, :]) < rc2
            hit &= members[None, :] != r[:, None]
            hit &= rank_m[None, :] <= RANK[tag[r]][:, None]
            b, m = np.nonzero(hit)                                # sources of each receiver
            d = x64[r[b]] - pm64[m]                               # FP64 r_ij
            dist = np.sqrt(np.einsum("pk,pk->p", d, d))
            t = np.clip(1.0 - 0.5 * dist / h, 0.0, None)
            w = K * t ** 3
            for k in range(3):
                a[rows, k] = np.bincount(b, weights=w * d[:, k], minlength=len(rows))
            S[rows] = np.bincount(b, weights=w * dist, minlength=len(rows))
            cnt[rows] = np.bincount(b, minlength=len(rows))
    return a, S, cnt


def amax_per_geometry(wl, a_all: np.ndarray, tag=None, gid=None) -> np.ndarray:
    """max over moving particles of |a_i| for every geometry (0 if none move)."""
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    mov = moving_mask(tag, wl.move_mask)
    out = np.zeros(len(wl.geoms))
    nrm = np.linalg.norm(a_all, axis=1)
    for g in range(len(wl.geoms)):
        m = mov & (gid == g)
        if m.any():
            out[g] = nrm[m].max()
    return out
