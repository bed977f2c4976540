"""The on-facet invariant at binary32 storage.

A surface particle is projected in FP64 onto its facet's plane and stored in
binary32: rounding each coordinate to nearest moves the point by at most half
an ulp per coordinate, so its distance from the plane is at most
0.5 sqrt(sum_c ulp(x_c)^2) (|n . e| <= |e| for a unit normal) on top of the
1e-6 dx of the strict invariant. This helper states that bound per particle,
from the particle's own stored coordinates.
"""
import numpy as np


def plane_distance(pos32, mesh, owner):
    """Distance of binary32 points from the planes of their owner facets (FP64)."""
    A, B, C = (mesh.vert[mesh.tri[owner, q]] for q in range(3))
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return np.abs(np.einsum("ij,ij->i", np.asarray(pos32, np.float64) - A, n))


def on_facet_bound(pos32, dx):
    """1e-6 dx + 0.5 |ulp(x)| per particle (ulp of each stored coordinate)."""
    ulp = np.spacing(np.abs(np.asarray(pos32, np.float32))).astype(np.float64)
    return 1e-6 * dx + 0.5 * np.linalg.norm(ulp, axis=1)


def assert_on_facets(pos32, mesh, owner, dx):
    d = plane_distance(pos32, mesh, owner)
    bound = on_facet_bound(pos32, dx)
    bad = d > bound
    assert not bad.any(), (f"{int(bad.sum())} particles off their facet: worst distance "
                           f"{float(d[bad].max()):.3g} (bound {float(bound[bad][np.argmax(d[bad])]):.3g})")
