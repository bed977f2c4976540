"""Pins of the three-layer volume split (oracle/band.py, section 3.3.4)
against closed forms: inside a convex box the distance to the surface is the
smallest distance to the six face planes; inside an icosphere it is 1 - |x| up
to the facets' sag."""
import numpy as np
import pytest

import synth
from oracle import band
from oracle import geometry
from synth import meshes as M

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_box_layers_match_plane_distances():
    wl = synth.cube_workload(n=12, seed=3)
    W = 2.5 / 12
    tag = band.layer_tags(wl, W)
    p = wl.pos.astype(np.float32).astype(np.float64)
    d = np.minimum(p, 1.0 - p).min(1)                      # closed form for the unit cube
    vol = wl.tag == synth.VOLUME
    clear = np.abs(d - W) > 1e-12
    assert np.array_equal(tag[vol & clear] == synth.FIXED, d[vol & clear] >= W)
    assert np.all(tag[vol & ~(d >= W)] == synth.VOLUME)
    # other classes keep their tags
    assert np.array_equal(tag[~vol], wl.tag[~vol])
    # both layers are populated
    assert (tag == synth.FIXED).sum() > 0 and ((tag == synth.VOLUME) & vol).sum() > 0


def test_width_limits():
    wl = synth.cube_workload(n=8, seed=4)
    vol = wl.tag == synth.VOLUME
    assert np.all(band.layer_tags(wl, 0.0)[vol] == synth.FIXED)        # every distance is >= 0
    assert np.all(band.layer_tags(wl, 10.0)[vol] == synth.VOLUME)      # nothing is that deep


def test_sphere_layers_within_facet_sag():
    wl = synth.sphere_workload(level=3, dx=0.1, seed=2)
    mesh = wl.geoms[0].mesh
    A, B, C, n = geometry.facet_frames(mesh.vert, mesh.tri)
    sag = 1.0 - np.min(np.einsum("ij,ij->i", n, A))
    W = 0.25
    tag = band.layer_tags(wl, W)
    r = np.linalg.norm(wl.pos.astype(np.float32).astype(np.float64), axis=1)
    vol = wl.tag == synth.VOLUME
    deep = vol & (1.0 - r >= W + sag)
    shallow = vol & (1.0 - r < W - sag)
    assert deep.any() and shallow.any()
    assert np.all(tag[deep] == synth.FIXED)
    assert np.all(tag[shallow] == synth.VOLUME)


def test_distance_to_single_facet_regions():
    """One triangle: a point over its interior is at the plane distance, one
    beyond a vertex at the vertex distance, one beside an edge at the edge
    distance (brute force over a fine sampling of the triangle agrees)."""
    vert = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    tri = np.array([[0, 1, 2]])
    pts = np.array([[0.2, 0.2, 0.3], [-0.5, -0.5, 0.1], [0.5, -0.4, 0.2], [1.5, 0.2, 0.0]])
    want = np.array([0.3, np.sqrt(0.5 + 0.01), np.sqrt(0.16 + 0.04), np.sqrt(0.25 + 0.04)])
    got = band.surface_distance(pts, vert, tri)
    assert np.allclose(got, want, atol=1e-14)
    s = np.linspace(0, 1, 401)
    u, v = np.meshgrid(s, s)
    keep = u + v <= 1
    samp = np.stack([u[keep], v[keep], np.zeros(keep.sum())], 1)
    brute = np.linalg.norm(pts[:, None, :] - samp[None], axis=-1).min(1)
    assert np.all(got <= brute + 1e-15) and np.all(brute - got < 2e-3)


def test_multi_geometry_uses_each_geometry_mesh():
    wl = synth.workload.solid_batch_workload(n_geom=3, n_min=2000, n_max=5000, seed=11)
    W = 2.0 * float(wl.geoms[0].dx)
    tag = band.layer_tags(wl, W)
    for g, geo in enumerate(wl.geoms):
        sel = np.flatnonzero((wl.gid == g) & (wl.tag == synth.VOLUME))
        d = geometry.unsigned_distance_many(wl.pos[sel].astype(np.float32).astype(np.float64),
                                            geo.mesh.vert, geo.mesh.tri)
        assert np.array_equal(tag[sel] == synth.FIXED, d >= W)
