"""Pins of the feature extraction (oracle/features.py, section 3.2.2): the
synthetic meshes carry their sharp edges by construction (from their
parametrisation, not from angles), so the extracted feature edges must be
exactly those; corner counts and the particle counts along straight edges
follow in closed form."""
import math

import numpy as np
import pytest

from oracle import features as F
from synth import meshes as M

COS30 = math.cos(math.radians(30.0))


def _constructed(m):
    return sorted({(int(min(a, b)), int(max(a, b))) for a, b in m.lines.seg_vert})


@pytest.mark.parametrize("name,make,n_sing", [("cube", M.cube, 8), ("cylinder", M.cylinder, 0),
                                               ("tetra", M.tetrahedron, 4),
                                               ("gear", lambda: M.gear(samples_per_period=12, rings=4), 192)])
def test_extracted_edges_are_the_constructed_sharp_edges(name, make, n_sing):
    m = make()
    fe = F.feature_edges(m.vert, m.tri, COS30)
    assert fe == _constructed(m)
    assert len(F.singular_vertices(fe)) == n_sing


def test_cube_lines_and_particles_closed_form():
    m = M.cube()
    dx = 0.05
    fe, sing, lines, closed, parts, sp = F.extract(m.vert, m.tri, COS30, dx)
    assert len(lines) == 12 and not any(closed)
    assert all(len(l) == 2 for l in lines)                      # every cube edge is one segment
    assert len(parts) == 12 * (math.ceil(1.0 / dx) - 1)
    assert np.allclose(sp, m.vert[sing])
    # spacing L/n along each edge
    for l in lines:
        a, b = m.vert[l[0]], m.vert[l[1]]
        on = np.abs(np.cross(parts - a, b - a)).sum(1) < 1e-12
        t = np.sort((parts[on] - a) @ (b - a))
        assert np.allclose(np.diff(np.concatenate([[0.0], t, [1.0]])), 1.0 / math.ceil(1.0 / dx))


def test_cylinder_rims_are_loops():
    m = M.cylinder(segments=64)
    dx = 0.03
    fe, sing, lines, closed, parts, sp = F.extract(m.vert, m.tri, COS30, dx)
    assert len(lines) == 2 and all(closed) and len(sing) == 0
    L = 64 * 2 * 0.5 * math.sin(math.pi / 64)
    assert len(parts) == 2 * math.ceil(L / dx)
    assert all(l[0] == min(l) for l in lines)
    r = np.linalg.norm(parts[:, :2], axis=1)   # on the 64-gon of radius 0.5
    assert np.all(r <= 0.5 + 1e-12) and np.all(r >= 0.5 * math.cos(math.pi / 64) - 1e-12)
    assert np.allclose(np.abs(parts[:, 2]), 0.5)


def test_threshold_limits():
    m = M.cube()
    assert F.feature_edges(m.vert, m.tri, 1.0) == _constructed(m)   # coplanar diagonals have n1.n2 = 1
    assert F.feature_edges(m.vert, m.tri, -1.0) == []                # nothing bends more than 180 degrees
