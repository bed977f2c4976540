"""Pins of the generation front end (oracle/generate.py; sections 3.1.1,
3.1.2, 3.2.1) against closed forms: for an axis-aligned box the cells meeting
its surface and the cells strictly inside it follow per axis from interval
arithmetic; an aligned grid with exact binary arithmetic exercises the ray
fill rule on shared facet edges; a box with a cavity must leave the cavity
out; on a sphere the classes agree with |c| up to the cell size and the sag."""
import numpy as np
import pytest

from oracle import generate as G
from synth import meshes as M


def _axis_counts(lo, hi, origin, dx, n):
    """Cells overlapping [lo, hi] (closed) and cells strictly inside (lo, hi)."""
    k = np.arange(n)
    a = origin + k * dx
    b = origin + (k + 1) * dx
    return int(np.sum((b >= lo) & (a <= hi))), int(np.sum((a > lo) & (b < hi)))


@pytest.mark.parametrize("lo,hi,dx", [((0.13, 0.21, 0.07), (0.87, 0.79, 0.93), 0.1),
                                       ((-0.31, 0.02, -0.44), (0.27, 0.61, 0.05), 0.07)])
def test_offset_box_classes_and_particles(lo, hi, dx):
    lo, hi = np.array(lo), np.array(hi)
    origin = lo - 2.3 * dx
    dims = np.ceil((hi - origin) / dx).astype(int) + 2
    m = M.cube(lo, hi)
    cls, pos, tag, owner = G.generate(m.vert, m.tri, dx, origin, dims)
    ov = [_axis_counts(lo[a], hi[a], origin[a], dx, dims[a]) for a in range(3)]
    n_over = ov[0][0] * ov[1][0] * ov[2][0]
    n_in = ov[0][1] * ov[1][1] * ov[2][1]
    assert int(np.sum(cls == G.INTERNAL)) == n_in
    assert int(np.sum(cls == G.SURFACE)) == n_over - n_in
    # one volume particle per internal cell, at its centre
    v = tag == G.VOLUME_TAG
    assert int(v.sum()) == n_in
    # surface particles lie on a face of the box, inside that face, on their owner facet's plane
    s = pos[tag == G.SURFACE_TAG]
    on_face = np.isclose(s, lo, atol=1e-12) | np.isclose(s, hi, atol=1e-12)
    assert np.all(on_face.any(1))
    assert np.all((s >= lo - 1e-12) & (s <= hi + 1e-12))
    A = m.vert[m.tri[owner[tag == G.SURFACE_TAG], 0]]
    n = np.cross(m.vert[m.tri[owner[tag == G.SURFACE_TAG], 1]] - A, m.vert[m.tri[owner[tag == G.SURFACE_TAG], 2]] - A)
    assert np.allclose(np.sum((s - A) * n, 1), 0.0, atol=1e-12)
    # every surface cell whose centre projects inside a face it meets gives a particle
    assert int((tag == G.SURFACE_TAG).sum()) <= n_over - n_in


def test_aligned_grid_fill_rule():
    """dx = 1/8 and origin -1/8: every coordinate is exact, facet edges (the
    face diagonals) pass through column centres, faces lie on cell faces."""
    m = M.cube()
    cls, pos, tag, owner = G.generate(m.vert, m.tri, 0.125, (-0.125,) * 3, (10, 10, 10))
    assert int(np.sum(cls == G.INTERNAL)) == 6 ** 3
    assert int(np.sum(cls == G.SURFACE)) == 10 ** 3 - 6 ** 3
    assert int(np.sum(cls == G.EXTERNAL)) == 0


def test_cavity_is_external():
    outer = M.cube((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    inner = M.cube((0.3, 0.3, 0.3), (0.7, 0.7, 0.7))
    vert = np.concatenate([outer.vert, inner.vert])
    tri = np.concatenate([outer.tri, inner.tri[:, ::-1] + len(outer.vert)])   # inner surface faces inwards
    dx = 0.1
    origin = np.full(3, -0.15)
    dims = (13, 13, 13)
    cls, _, _, _ = G.generate(vert, tri, dx, origin, dims)
    c = origin[0] + (np.arange(13) + 0.5) * dx
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    in_outer = (X > 0.05) & (X < 0.95) & (Y > 0.05) & (Y < 0.95) & (Z > 0.05) & (Z < 0.95)
    in_cavity = (X > 0.25) & (X < 0.75) & (Y > 0.25) & (Y < 0.75) & (Z > 0.25) & (Z < 0.75)
    # centres at least half a cell from both surfaces: classes follow from the nesting
    far = in_outer & ~((X > 0.25 - 1e-9) & (X < 0.75 + 1e-9) & (Y > 0.25 - 1e-9) & (Y < 0.75 + 1e-9)
                       & (Z > 0.25 - 1e-9) & (Z < 0.75 + 1e-9))
    assert np.all(cls[far] == G.INTERNAL)
    deep = (X > 0.35) & (X < 0.65) & (Y > 0.35) & (Y < 0.65) & (Z > 0.35) & (Z < 0.65)
    assert deep.any() and np.all(cls[deep] == G.EXTERNAL)
    assert np.all(cls[in_cavity & (cls != G.SURFACE)] == G.EXTERNAL)


def test_sphere_classes_follow_radius():
    m = M.icosphere(3)
    A = m.vert[m.tri[:, 0]]
    n = np.cross(m.vert[m.tri[:, 1]] - A, m.vert[m.tri[:, 2]] - A)
    n /= np.linalg.norm(n, axis=1)[:, None]
    sag = 1.0 - np.min(np.sum(n * A, 1))
    dx = 0.1
    origin = np.full(3, -1.25)
    dims = (25, 25, 25)
    cls, pos, tag, owner = G.generate(m.vert, m.tri, dx, origin, dims)
    c = origin[0] + (np.arange(25) + 0.5) * dx
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    half_diag = 0.5 * np.sqrt(3) * dx
    assert np.all(cls[r < 1.0 - sag - half_diag] == G.INTERNAL)
    assert np.all(cls[r > 1.0 + half_diag] == G.EXTERNAL)
    s = pos[tag == G.SURFACE_TAG]
    assert np.all(np.abs(np.linalg.norm(s, axis=1) - 1.0) <= sag + 1e-12)


def test_triangle_box_overlap_cases():
    """A facet touching a box face counts; one just beyond it does not; a
    facet cutting the box diagonally without any vertex inside counts."""
    c = np.zeros(3)
    hw = np.full(3, 0.5)
    a, b, cc = np.array([0.5, -1, -1.0]), np.array([0.5, 2, -1.0]), np.array([0.5, -1, 2.0])
    assert G.tri_box_overlap(c, hw, a, b, cc)
    eps = np.array([1e-12, 0, 0])
    assert not G.tri_box_overlap(c, hw, a + eps, b + eps, cc + eps)
    # a large triangle in the plane x + y + z = 0 through the box, vertices far outside
    a, b, cc = np.array([5.0, -5, 0]), np.array([0.0, 5, -5]), np.array([-5.0, 0, 5])
    assert G.tri_box_overlap(c, hw, a, b, cc)
    # the same plane shifted beyond the box corner (|x + y + z| > 1.5)
    sh = np.full(3, 0.51)
    assert not G.tri_box_overlap(c, hw, a + sh, b + sh, cc + sh)


def _classes(lo, hi, dx, origin, dims):
    m = M.cube(lo, hi)
    return G.classify(m.vert, m.tri, dx, np.asarray(origin, np.float64), dims)


def test_boolean_of_boxes_matches_the_combined_box():
    """Axis-aligned boxes whose intersection, difference and union are boxes:
    the internal cells of the combination are those of the combined box."""
    dx, origin, dims = 0.1, (-0.05, -0.05, -0.05), (24, 14, 14)
    A = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    B = ((0.53, 0.0 - 0.2, 0.0 - 0.2), (2.03, 1.2, 1.2))       # covers A beyond x = 0.53 in y and z
    ca, cb = _classes(*A, dx, origin, dims), _classes(*B, dx, origin, dims)
    inter = _classes((0.53, 0.0, 0.0), (1.0, 1.0, 1.0), dx, origin, dims)
    diff = _classes((0.0, 0.0, 0.0), (0.53, 1.0, 1.0), dx, origin, dims)
    assert np.array_equal(G.boolean(ca, cb, G.INTERSECTION) == G.INTERNAL, inter == G.INTERNAL)
    assert np.array_equal(G.boolean(ca, cb, G.DIFFERENCE) == G.INTERNAL, diff == G.INTERNAL)
    # union with a box that extends A along x through a thick overlap
    C = ((0.47, 0.0, 0.0), (2.03, 1.0, 1.0))
    cc = _classes(*C, dx, origin, dims)
    uni = _classes((0.0, 0.0, 0.0), (2.03, 1.0, 1.0), dx, origin, dims)
    assert np.array_equal(G.boolean(ca, cc, G.UNION) == G.INTERNAL, uni == G.INTERNAL)
    # the combined surface cells cover the combined box's surface cells
    for op, box in ((G.INTERSECTION, inter), (G.DIFFERENCE, diff)):
        got = G.boolean(ca, cb, op)
        assert np.all(got[box == G.SURFACE] == G.SURFACE)
    assert np.all(G.boolean(ca, cc, G.UNION)[uni == G.SURFACE] != G.EXTERNAL)


def test_boolean_identities():
    dx, origin, dims = 0.1, (-0.15, -0.15, -0.15), (14, 14, 14)
    ca = _classes((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), dx, origin, dims)
    empty = np.zeros_like(ca)
    assert np.array_equal(G.boolean(ca, ca, G.UNION), ca)
    assert np.array_equal(G.boolean(ca, ca, G.INTERSECTION), ca)
    assert np.array_equal(G.boolean(ca, empty, G.UNION), ca)
    assert np.array_equal(G.boolean(ca, empty, G.DIFFERENCE), ca)
    assert not np.any(G.boolean(ca, ca, G.DIFFERENCE) == G.INTERNAL)
