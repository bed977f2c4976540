"""Feature extraction on the GPU (fppg_features, section 3.2.2) against the
oracle: feature edges, singular vertices and lines exactly, feature-line
particles as the binary32 of the oracle's FP64 points."""
import math

import numpy as np
import pytest

from oracle import features as F
from synth import meshes as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

COS30 = math.cos(math.radians(30.0))


def _features(vert, tri, c, dx):
    from paper_2501_03056_amd.front import features
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = features(vert, tri, c, dx)
    return {k: v.cpu().numpy() for k, v in out.items()}


CASES = {
    "cube": (lambda: M.cube(), 0.05),
    "cylinder": (lambda: M.cylinder(segments=64), 0.03),
    "tetra": (lambda: M.tetrahedron(), 0.04),
    "gear_coarse": (lambda: M.gear(samples_per_period=12, rings=4), 0.02),
    "gear": (lambda: M.gear(), 0.004),
    "sphere": (lambda: M.icosphere(3), 0.05),
}


@pytest.mark.parametrize("case", list(CASES))
def test_features_match_oracle(case):
    make, dx = CASES[case]
    m = make()
    got = _features(m.vert, m.tri, COS30, dx)
    fe, sing, lines, closed, parts, _ = F.extract(m.vert, m.tri, COS30, dx)
    assert [tuple(e) for e in got["edges"].tolist()] == fe
    assert got["singular"].tolist() == sing
    lb = got["line_begin"]
    glines = [got["line_vert"][lb[i]:lb[i + 1]].tolist() for i in range(len(lb) - 1)]
    assert glines == lines
    assert got["line_closed"].tolist() == closed
    assert len(got["pos"]) == len(parts)
    assert np.array_equal(got["pos"][:, :3], parts.astype(np.float32))
    assert np.all(got["pos"][:, 3].view(np.int32) == 1)


def test_open_mesh_boundary_edges_are_features():
    """A single square of two triangles: its four boundary edges form one loop
    (no vertex on more than two of them); the diagonal is flat."""
    vert = np.array([[0.0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]])
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    got = _features(vert, tri, COS30, 0.25)
    fe, sing, lines, closed, parts, _ = F.extract(vert, tri, COS30, 0.25)
    assert [tuple(e) for e in got["edges"].tolist()] == fe == [(0, 1), (0, 3), (1, 2), (2, 3)]
    assert got["line_closed"].tolist() == closed == [1]
    assert np.array_equal(got["pos"][:, :3], parts.astype(np.float32))


def test_particle_segment_and_arc_are_consistent():
    m = M.gear(samples_per_period=12, rings=4)
    got = _features(m.vert, m.tri, COS30, 0.02)
    lb, lv = got["line_begin"], got["line_vert"]
    closed = got["line_closed"]
    for k in range(0, len(got["pos"]), 7):
        l, s, u = int(got["line_of"][k]), int(got["seg"][k]), float(got["u"][k])
        vs = lv[lb[l]:lb[l + 1]].tolist() + ([lv[lb[l]]] if closed[l] else [])
        a, b = m.vert[vs[s]], m.vert[vs[s + 1]]
        L = np.linalg.norm(b - a)
        assert -1e-12 <= u <= L + 1e-12
        before = sum(np.linalg.norm(m.vert[vs[i + 1]] - m.vert[vs[i]]) for i in range(s))
        assert abs(before + u - got["arc"][k]) < 1e-12
        assert np.allclose(got["pos"][k, :3], (a + (u / L) * (b - a)).astype(np.float32), atol=1e-6)
