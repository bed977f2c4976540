"""Three-layer volume relaxation (section 3.3.4), in FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the product path never imports it.

The paper splits the volume particles into two layers beneath the surface
particles: an intermediate layer next to the surface, which is relaxed, and an
innermost core, which is not; the core particles act as sources for the
intermediate ones (they keep the intermediate layer from leaking inwards) and
the surface particles act as sources from outside. The width of the layers is
a user parameter.

Reading (the paper gives the layers by a user-defined width, not by a
formula): a volume particle belongs to the intermediate layer iff the exact
unsigned distance from its binary32 position to its geometry's surface mesh
is below the width W; every other volume particle becomes a fixed particle
(tag FIXED). The distance is the minimum over all facets of the point-triangle
distance (oracle.geometry, Voronoi-region closest point), evaluated in FP64;
the decision compares squared distances with W^2.
"""
import numpy as np

from . import geometry

VOLUME, FIXED = 3, 4


def layer_tags(wl, width: float, gid=None) -> np.ndarray:
    """New tag array of the workload: volume particles at distance >= width
    from their geometry's surface mesh are re-tagged FIXED."""
    tag = np.asarray(wl.tag, np.int32).copy()
    gid = np.asarray(wl.gid if gid is None else gid)
    pos = np.asarray(wl.pos, np.float32).astype(np.float64)
    for g, geo in enumerate(wl.geoms):
        sel = np.flatnonzero((tag == VOLUME) & (gid == g))
        if not len(sel):
            continue
        d = surface_distance(pos[sel], geo.mesh.vert, geo.mesh.tri)
        tag[sel[d * d >= width * width]] = FIXED
    return tag


def surface_distance(p: np.ndarray, vert, tri) -> np.ndarray:
    """Unsigned distance of points [P, 3] to the facets of a mesh (FP64)."""
    return geometry.unsigned_distance_many(np.asarray(p, np.float64), vert, tri)
