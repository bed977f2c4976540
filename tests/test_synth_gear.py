"""The synthetic 24-tooth gear workload: every particle class sits where its
definition puts it (CPU, coarse spacing)."""
import numpy as np
import pytest

import synth
from oracle import geometry as ogeo


@pytest.fixture(scope="module")
def gear():
    return synth.gear_workload(dx=0.02, seed=3)


def test_gear_mesh_and_counts(gear):
    mesh = gear.geoms[0].mesh
    assert mesh.n_tri == 2 * 35 * 1440 * 2 + 2 * 1440 * 2          # 207,360 facets
    assert len(mesh.singular) == 192
    c = gear.counts()
    assert c["singular"] == 192 and c["feature"] > 0 and c["surface"] > 0 and c["volume"] > 0


def test_surface_particles_lie_in_their_facets(gear):
    mesh = gear.geoms[0].mesh
    s = np.nonzero(gear.tag == synth.SURFACE)[0]
    f = gear.owner[s]
    A, B, C = (mesh.vert[mesh.tri[f, q]] for q in range(3))
    p = gear.pos[s].astype(np.float64)
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    assert np.abs(np.einsum("ij,ij->i", p - A, n)).max() < 1e-6
    la, lb, lc = ogeo.barycentric(p, A, B, C)
    assert min(la.min(), lb.min(), lc.min()) > -1e-5


def test_feature_and_singular_particles_on_their_lines(gear):
    lines = gear.geoms[0].mesh.lines
    f = np.nonzero(gear.tag == synth.FEATURE)[0]
    slot = gear.owner[f]
    seg = gear.feat_seg[slot]
    p0, p1 = lines.seg_p[seg, 0], lines.seg_p[seg, 1]
    t = (p1 - p0) / np.linalg.norm(p1 - p0, axis=1, keepdims=True)
    want = p0 + gear.feat_u[slot][:, None] * t
    assert np.abs(gear.pos[f] - want).max() < 1e-6
    s = gear.tag == synth.SINGULAR
    mesh = gear.geoms[0].mesh
    assert np.array_equal(gear.pos[s], mesh.vert[gear.owner[s]].astype(np.float32))


def test_volume_particles_are_half_a_spacing_inside():
    wl = synth.gear_workload(dx=0.04, seed=3)
    mesh = wl.geoms[0].mesh
    v = np.nonzero(wl.tag == synth.VOLUME)[0]
    sel = np.random.Generator(np.random.PCG64(0)).choice(v, 12, replace=False)
    sd = ogeo.signed_distance_many(wl.pos[sel].astype(np.float64), mesh.vert, mesh.tri)
    assert np.all(sd <= -0.5 * 0.04 * (1 - 1e-3))
