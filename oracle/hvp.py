"""Jacobian of the relaxation force field and the pair energy it derives from.

Not in the paper (an addition for Newton-Krylov relaxation and gradients).
With f(r) = K (1 - |r|/2h)^3 r the pair term of Eq. 15 (force.py),

    M(r) = df/dr = K [ t^3 I - (3/(2h)) t^2 r r^T / |r| ],   t = 1 - |r|/(2h)

(finite as r -> 0). For moving receiver i with sources src(i):
    (J v)_i = sum_{j in src(i)} M(r_ij) (v_i - v_j)
and (J v)_i = 0 for non-moving i. The transpose product is
    (J^T u)_k = [sum_{j in src(k)} M(r_kj)] u_k  -  sum_{i moving, k in src(i)} M(r_ik) u_i .
When the moving particles all share one rank and every other source is fixed,
a = -grad E with
    E = 1/2 sum_{i, j both moving, j in src(i)} W(r_ij) + sum_{i moving, j fixed source} W(r_ij)
and J = -Hess(E) is symmetric.
"""
import numpy as np

from . import force as F
from .kernel import W, force_coef
from .neighbors import pair_d2, rc2_f32


def _pairs(wl, pos32, tag, gid):
    """All (receiver i, source j) pairs of moving receivers, with FP64 r_ij and h."""
    mov = F.moving_mask(tag, wl.move_mask)
    I, J, H = [], [], []
    for g, geo in enumerate(wl.geoms):
        members = np.nonzero(gid == g)[0]
        rc2 = rc2_f32(geo.h)
        rank_m = F.RANK[tag[members]]
        rec = members[mov[members]]
        step = max(1, (1 << 24) // max(len(members), 1))
        for s in range(0, len(rec), step):
            r = rec[s:s + step]
            hit = pair_d2(pos32[r][:, None, :], pos32[members][None, :, :]) < rc2
            hit &= members[None, :] != r[:, None]
            hit &= rank_m[None, :] <= F.RANK[tag[r]][:, None]
            b, m = np.nonzero(hit)
            I.append(r[b])
            J.append(members[m])
            H.append(np.full(len(b), float(geo.h)))
    if not I:
        return np.zeros(0, int), np.zeros(0, int), np.zeros(0)
    return np.concatenate(I), np.concatenate(J), np.concatenate(H)


def pair_jacobian(r: np.ndarray, h: np.ndarray) -> np.ndarray:
    """M(r) for pair vectors r [P, 3] -> [P, 3, 3]."""
    d = np.linalg.norm(r, axis=1)
    t = np.clip(1.0 - d / (2.0 * h), 0.0, None)
    K = force_coef(1.0) / h ** 5          # force_coef(h) = force_coef(1) / h^5
    safe = np.where(d > 0, d, 1.0)
    rr = np.einsum("pi,pj->pij", r, r) / safe[:, None, None]
    eye = np.eye(3)[None]
    return K[:, None, None] * (t[:, None, None] ** 3 * eye
                               - (3.0 / (2.0 * h))[:, None, None] * t[:, None, None] ** 2 * rr)


def jvp(wl, v, pos32=None, tag=None, gid=None, pos64=None):
    """(J v) for v [N, 3] (pair vectors from pos64 when given, see force.accel)."""
    pos32 = wl.pos if pos32 is None else pos32
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    I, J, H = _pairs(wl, pos32, tag, gid)
    x = pos32.astype(np.float64) if pos64 is None else np.asarray(pos64, np.float64)
    M = pair_jacobian(x[I] - x[J], H)
    contrib = np.einsum("pij,pj->pi", M, v[I] - v[J])
    out = np.zeros_like(np.asarray(v, np.float64))
    for k in range(3):
        out[:, k] = np.bincount(I, weights=contrib[:, k], minlength=len(x))
    return out


def vjp(wl, u, pos32=None, tag=None, gid=None):
    """(J^T u) for u [N, 3]."""
    pos32 = wl.pos if pos32 is None else pos32
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    I, J, H = _pairs(wl, pos32, tag, gid)
    x = pos32.astype(np.float64)
    M = pair_jacobian(x[I] - x[J], H)
    Mu = np.einsum("pij,pj->pi", M, u[I])      # M symmetric
    out = np.zeros_like(np.asarray(u, np.float64))
    for k in range(3):
        out[:, k] = np.bincount(I, weights=Mu[:, k], minlength=len(x))
        out[:, k] -= np.bincount(J, weights=Mu[:, k], minlength=len(x))
    return out


def energy(wl, pos64, tag=None, gid=None):
    """Pair energy E of the moving set (single moving rank, fixed other sources),
    evaluated at FP64 positions with the neighbour set of their binary32 rounding."""
    tag = wl.tag if tag is None else tag
    gid = wl.gid if gid is None else gid
    pos32 = np.asarray(pos64, np.float64).astype(np.float32)
    I, J, H = _pairs(wl, pos32, tag, gid)
    mov = F.moving_mask(tag, wl.move_mask)
    d = np.linalg.norm(pos64[I] - pos64[J], axis=1)
    w = np.array([W(di, hi) for di, hi in zip(d, H)]) if len(d) < 64 else W(d, H)
    weight = np.where(mov[J], 0.5, 1.0)
    return float(np.sum(weight * w))
