"""Neighbour predicate, evaluated by brute force over all pairs.

The paper sums over the particles inside the kernel support (Eq. 15-16: q <= 2,
i.e. r <= r_c = 2h) but does not fix the arithmetic of the test. Reading: the
test is one fixed binary32 expression, so that a GPU and a CPU can agree on it
exactly. For particles i != j of the same geometry:

    ddx = fl32(x_i - x_j)  (and y, z)
    d2  = fl32(fl32(fl32(ddx*ddx) + fl32(ddy*ddy)) + fl32(ddz*ddz))
    neighbour  <=>  d2 < rc2,   rc2 = fl32(fl32(2h) * fl32(2h))

numpy float32 arithmetic rounds each elementwise operation separately (no
fused multiply-add), which is exactly this definition.
"""
import numpy as np


def rc2_f32(h: float) -> np.float32:
    rc = np.float32(2.0) * np.float32(h)
    return np.float32(rc * rc)


def pair_d2(pi: np.ndarray, pj: np.ndarray) -> np.ndarray:
    """binary32 squared distance of broadcastable position arrays [..., 3]."""
    pi = np.asarray(pi, np.float32)
    pj = np.asarray(pj, np.float32)
    acc = pair_d2_xyz(pi[..., 0], pi[..., 1], pi[..., 2], pj[..., 0], pj[..., 1], pj[..., 2])
    return acc if acc.shape == np.broadcast_shapes(pi.shape, pj.shape)[:-1] else acc.reshape(())


def pair_d2_xyz(xi, yi, zi, xj, yj, zj) -> np.ndarray:
    """The same binary32 squared distance from coordinate arrays (broadcastable)."""
    acc = None
    for a, b in ((xi, xj), (yi, yj), (zi, zj)):   # ((ddx^2 + ddy^2) + ddz^2), each op rounded
        d = np.atleast_1d(np.subtract(a, b, dtype=np.float32))
        np.multiply(d, d, out=d)
        if acc is None:
            acc = d
        else:
            np.add(acc, d, out=acc)
    return acc


def neighbor_lists(wl, receivers=None, pos32=None, chunk=256):
    """For each receiver index i: ascending array of j with pred(i, j), all tags.

    Brute force: every receiver is tested against every particle of its
    geometry.
    """
    pos32 = wl.pos if pos32 is None else pos32
    receivers = np.arange(wl.n) if receivers is None else np.asarray(receivers)
    out = {}
    for g, geo in enumerate(wl.geoms):
        members = np.nonzero(wl.gid == g)[0]
        pm = pos32[members]
        rc2 = rc2_f32(geo.h)
        rec = receivers[wl.gid[receivers] == g]
        for s in range(0, len(rec), chunk):
            r = rec[s:s + chunk]
            d2 = pair_d2(pos32[r][:, None, :], pm[None, :, :])
            hit = d2 < rc2
            hit &= members[None, :] != r[:, None]
            for a, i in enumerate(r):
                out[int(i)] = members[hit[a]]
    return out
