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


def test_capacity_error_keeps_the_sizes():
    """Outputs one particle short: E_CAPACITY, nothing written, and the counts
    still hold the sizes needed."""
    import ctypes
    from paper_2501_03056_amd import _lib as L
    from paper_2501_03056_amd.relax import Context
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = M.cube()
    ctx = Context(0)
    vert = np.ascontiguousarray(m.vert, np.float64)
    tri = np.ascontiguousarray(m.tri, np.int32)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(o):
        return ctx.lib.fppg_features(ctx.handle, vert.ctypes.data_as(ctypes.c_void_p), len(vert),
                                     tri.ctypes.data_as(ctypes.c_void_p), len(tri), COS30, 0.05, ctypes.byref(o),
                                     stream)

    sizes = L.FeaturesOut()
    assert call(sizes) == L.OK
    assert (sizes.n_edges, sizes.n_singular, sizes.n_lines) == (12, 8, 12)
    np_ = sizes.n_particles
    d = "cuda"
    edges = torch.empty((12, 2), dtype=torch.int32, device=d)
    sing = torch.empty(8, dtype=torch.int32, device=d)
    lb = torch.full((13,), -7, dtype=torch.int32, device=d)
    lv = torch.empty(sizes.n_line_vert, dtype=torch.int32, device=d)
    lc = torch.empty(12, dtype=torch.uint8, device=d)
    pos = torch.empty((np_, 4), dtype=torch.float32, device=d)
    li = torch.empty(np_, dtype=torch.int32, device=d)
    arc = torch.empty(np_, dtype=torch.float64, device=d)
    seg = torch.empty(np_, dtype=torch.int32, device=d)
    u = torch.empty(np_, dtype=torch.float64, device=d)
    P = L.ptr
    o = L.FeaturesOut(P(edges), 12, P(sing), 8, P(lb), P(lv), P(lc), 12, sizes.n_line_vert, P(pos), P(li), P(arc),
                      P(seg), P(u), np_ - 1)
    assert call(o) == L.E_CAPACITY
    assert o.n_particles == np_ and o.n_edges == 12
    assert (lb == -7).all()
    o.cap_particles = np_
    assert call(o) == L.OK
    torch.cuda.synchronize()
    assert lb[-1].item() == sizes.n_line_vert
    ctx.close()
