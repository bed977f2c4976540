"""Boolean assemblies in the oracle (section 3.2.3 combines solids by Boolean
operations; the paper shows it for the background-grid cells only).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

An assembly is the union of closed parts, or part 0 minus the union of the
others; its facets are those of the parts. Reading (the paper states no rule
for relaxing on a combined surface; parity unpinned as a reading):

  part signed distance   sd_k(p) = winding-number sign of part k's facets
                         (geometry.winding_number) times the exact distance to
                         them (geometry.unsigned_distance_many)
  assembly               sd(p) = min_k sd_k(p)                       (union)
                         sd(p) = max(sd_0(p), -min_{k>=1} sd_k(p))   (difference)
  surface projection     a foot point p on a facet of part k counts only where
                         it lies on the assembly's boundary: union, outside or
                         on every other part (sd_j(p) >= 0); difference, for
                         k = 0 outside or on every cut part, for a cut part k
                         inside or on part 0 (sd_0(p) <= 0) and outside or on
                         the other cut parts
  volume rule            accepted iff sd(y) < 0, as for a single mesh
  margins                a foot within 1e-9 of another part's surface, where
                         its membership could flip under rounding
"""
import numpy as np

from .geometry import unsigned_distance_many, winding_number

UNION, DIFFERENCE = 1, 2


def part_sd(p, vert, tri):
    """Signed distance of points p [P, 3] to one closed part (negative inside)."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    if len(p) == 0:
        return np.zeros(0)
    wn = winding_number(p, vert, tri)
    d = unsigned_distance_many(p, vert, tri)
    return np.where(wn > 0.5, -d, d)


def parts_sd(p, geo):
    """sd_k(p) for every part k of the assembly: [P, n_part]."""
    c = geo.csg
    tb = c.part_tri_begin
    return np.stack([part_sd(p, geo.mesh.vert, geo.mesh.tri[tb[k]:tb[k + 1]]) for k in range(c.n_part)], 1)


def assembly_sd(p, geo):
    sd = parts_sd(p, geo)
    if geo.csg.op == UNION:
        return sd.min(1)
    rest = sd[:, 1:].min(1) if sd.shape[1] > 1 else np.full(len(sd), np.inf)
    return np.maximum(sd[:, 0], -rest)


def part_of_facets(geo, facets):
    """Part index of local facet indices."""
    return np.searchsorted(geo.csg.part_tri_begin, facets, side="right") - 1


def on_boundary(p, facets, geo, margin=1e-9):
    """For foot points p [P, 3] on local facets `facets` [P]: (on the assembly's
    boundary, within `margin` of deciding part surfaces)."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    if len(p) == 0:
        return np.zeros(0, bool), np.zeros(0, bool)
    sd = parts_sd(p, geo)
    k = part_of_facets(geo, np.asarray(facets))
    ok = np.ones(len(p), bool)
    near = np.zeros(len(p), bool)
    for j in range(geo.csg.n_part):
        other = k != j
        if geo.csg.op == DIFFERENCE and j == 0:
            cond = np.where(k > 0, sd[:, 0] <= 0.0, True)
            dec = k > 0
        else:
            cond = sd[:, j] >= 0.0
            dec = other & ~((geo.csg.op == DIFFERENCE) & (k > 0) & (j == 0))
        ok &= np.where(other, cond, True)
        near |= dec & other & (np.abs(sd[:, j]) <= margin)
    return ok, near
