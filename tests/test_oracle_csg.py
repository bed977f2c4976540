"""Pins of the oracle's Boolean assemblies (oracle/csg.py) against boxes whose
union or difference is again a box, where the answer is the box's own:

  * the sign of the assembly's signed distance equals the combined box's
  * the surface projection lands on the combined box's faces, never on a
    part's face inside the other part
  * the full-size mode decides every particle of an assembly batch as the
    brute-force step does
and of the clipped sharp edges of the inputs (a cylinder cut by a box).
"""
import math

import numpy as np
import pytest

import synth
from synth import csg as C
from synth import meshes as M
from oracle import csg, force, local, step


def _geo(parts, op, dx=0.05):
    mesh, info, _ = C.combine(parts, op)
    geo = synth.workload._make_geom(mesh, dx)
    geo.csg = info
    return geo


def _box_sd(p, lo, hi):
    lo, hi = np.asarray(lo), np.asarray(hi)
    q = np.maximum(lo - p, p - hi)
    out = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    return np.where(np.all(q < 0, axis=1), q.max(1), out)


CASES = {
    # [0,1]^3 u [0.5,1.5]x[0,1]^2 = [0,1.5]x[0,1]^2
    "union": ([((0, 0, 0), (1, 1, 1)), ((0.5, 0, 0), (1.5, 1, 1))], C.UNION, ((0, 0, 0), (1.5, 1, 1))),
    # [0,1]^3 minus [0.5,2]x[-1,2]^2 = [0,0.5]x[0,1]^2
    "difference": ([((0, 0, 0), (1, 1, 1)), ((0.5, -1, -1), (2, 2, 2))], C.DIFFERENCE, ((0, 0, 0), (0.5, 1, 1))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_assembly_sign_is_the_combined_box(case):
    boxes, op, (lo, hi) = CASES[case]
    geo = _geo([M.cube(a, b) for a, b in boxes], op)
    rng = np.random.Generator(np.random.PCG64(3))
    p = rng.uniform(-0.3, 1.8, size=(4000, 3))
    ref = _box_sd(p, lo, hi)
    far = np.abs(ref) > 1e-6
    got = csg.assembly_sd(p[far], geo)
    assert np.array_equal(got < 0, ref[far] < 0)


@pytest.mark.parametrize("case", list(CASES))
def test_projection_lands_on_the_combined_box(case):
    """Points just off a face of the combined box project onto that face
    (foot = the point with its normal coordinate set to the face's); points
    just off a part's face that lies inside the assembly find no facet."""
    boxes, op, (lo, hi) = CASES[case]
    geo = _geo([M.cube(a, b) for a, b in boxes], op, dx=0.05)
    R = float(geo.proj_radius)
    rng = np.random.Generator(np.random.PCG64(4))
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    pts, want = [], []
    for _ in range(300):
        ax = int(rng.integers(3))
        side = int(rng.integers(2))
        q = rng.uniform(lo + 0.1, hi - 0.1)
        q[ax] = (hi if side else lo)[ax] + rng.uniform(-0.5, 0.5) * R
        w = q.copy()
        w[ax] = (hi if side else lo)[ax]
        pts.append(q)
        want.append(w)
    pts, want = np.array(pts), np.array(want)
    wl_like = type("W", (), {"geoms": [geo]})()
    ok, foot, own, margin = step.project_surface(wl_like, pts, 0)
    # in the union the two boxes share the strip 0.5 <= x <= 1 of their y and z
    # faces: there a foot lies on both parts' surfaces and membership is decided
    # by rounding; the oracle flags those feet as margin cases
    shared = (want[:, 0] >= 0.5 - 1e-9) & (want[:, 0] <= 1.0 + 1e-9) & (np.abs(want[:, 0] - 1.5) > 1e-9) \
        if case == "union" else np.zeros(len(want), bool)
    assert margin[shared].all()
    assert ok[~shared].all()
    assert np.abs(foot[~shared] - want[~shared]).max() <= 1e-12
    # a part's face inside the assembly: union, part 0's face x = 1 inside part 1;
    # difference, part 1's face x = 2 outside part 0
    inner_x = 1.0 if case == "union" else 2.0
    q = np.column_stack([np.full(50, inner_x + 0.3 * R), rng.uniform(0.3, 0.7, 50), rng.uniform(0.3, 0.7, 50)])
    ok, _, _, _ = step.project_surface(wl_like, q, 0)
    assert not ok.any()


def test_clipped_rim_of_a_cut_cylinder():
    """A cylinder of radius 0.5 minus the half-space x > 0.2 (a large box): both
    rim loops become one open line each, outside the box, of the length of the
    64-gon's arc with x < 0.2."""
    cyl = M.cylinder(0.5, 1.0, 64)
    cut = M.cube((0.2, -1, -1), (2, 1, 1))
    mesh, info, parts_P = C.combine([cyl, cut], C.DIFFERENCE, with_curves=False)
    L = mesh.lines
    assert L.n_line == 2 and not L.line_closed.any()
    p = L.seg_p.reshape(-1, 3)
    assert p[:, 0].max() <= 0.2 + 1e-12
    th = np.arange(65) * 2 * np.pi / 64
    ring = np.stack([0.5 * np.cos(th), 0.5 * np.sin(th)], 1)
    # arc length of the polygon with x <= 0.2, clipping the two crossing edges
    length = 0.0
    for a, b in zip(ring[:-1], ring[1:]):
        if a[0] <= 0.2 and b[0] <= 0.2:
            length += np.linalg.norm(b - a)
        elif (a[0] - 0.2) * (b[0] - 0.2) < 0:
            t = (0.2 - a[0]) / (b[0] - a[0])
            c = a + t * (b - a)
            length += np.linalg.norm(c - (a if a[0] <= 0.2 else b))
    for l in range(2):
        s0, s1 = L.line_seg_begin[l], L.line_seg_begin[l + 1]
        got = np.linalg.norm(L.seg_p[s0:s1, 1] - L.seg_p[s0:s1, 0], axis=1).sum()
        assert got == pytest.approx(length, rel=1e-12)
    assert math.isfinite(length)


@pytest.mark.parametrize("boxes,op,length,loops", [
    # [0,1]^3 minus [0.5,2]x[-1,2]^2: the cut face x = 0.5 meets the box's four faces
    ([((0, 0, 0), (1, 1, 1)), ((0.5, -1, -1), (2, 2, 2))], C.DIFFERENCE, 4.0, 1),
    # corner-overlapping cubes: six half-edges around the shared corner region
    ([((0, 0, 0), (1, 1, 1)), ((0.5, 0.5, 0.5), (1.5, 1.5, 1.5))], C.UNION, 3.0, 1),
    ([((0, 0, 0), (1, 1, 1)), ((0.5, 0.5, 0.5), (1.5, 1.5, 1.5))], C.DIFFERENCE, 3.0, 1),
    # a union that is again a box has no crease between the parts
    ([((0, 0, 0), (1, 1, 1)), ((0.5, 0, 0), (1.5, 1, 1))], C.UNION, 0.0, 0),
])
def test_intersection_curves_of_boxes(boxes, op, length, loops):
    """The curves where the parts' faces meet on the assembly's boundary at a
    crease, by hand; every point of them on the assembly's surface."""
    parts = [M.cube(a, b) for a, b in boxes]
    P = [C.planes(p) for p in parts]
    polys, closed = C.intersection_lines(op, parts, P)
    got = sum(np.linalg.norm(np.diff(np.asarray(pl), axis=0), axis=1).sum() for pl in polys)
    assert got == pytest.approx(length, abs=1e-12)
    assert sum(closed) == loops and all(closed)
    if polys:
        pts = np.concatenate([np.asarray(pl) for pl in polys])
        geo = _geo(parts, op)
        assert np.abs(csg.assembly_sd(pts, geo)).max() < 1e-12


def test_assembly_lines_run_between_singular_points():
    """With the curves, every open line of an assembly starts and ends at a
    singular point and none passes through one."""
    rng = np.random.Generator(np.random.PCG64(4001))
    parts, op, _ = C.random_assembly(rng, 50_000)
    mesh, info, _ = C.combine(parts, op)
    L = mesh.lines
    S = mesh.singular
    tol = 1e-9 * max(np.ptp(p.vert, 0).max() for p in parts)
    for l in range(L.n_line):
        s0, s1 = L.line_seg_begin[l], L.line_seg_begin[l + 1]
        pts = np.concatenate([L.seg_p[s0:s1, 0], L.seg_p[s1 - 1:s1, 1]])
        d = np.linalg.norm(pts[:, None, :] - S[None], axis=2).min(1) if len(S) else np.full(len(pts), np.inf)
        if L.line_closed[l]:
            assert (d > tol).all()
        else:
            assert d[0] <= tol and d[-1] <= tol and (d[1:-1] > tol).all()


def test_full_size_mode_on_an_assembly_batch():
    wl = synth.workload.batch_workload(n_geom=3, n_min=1.5e3, n_max=3e3, seed=4100, mc_samples=100_000)
    ref = step.relax_step(wl)
    got = local.relax_step(wl)
    assert np.array_equal(ref.reverted, got.reverted)
    assert np.array_equal(ref.margin, got.margin)
    assert np.array_equal(ref.owner, got.owner)
    assert np.allclose(ref.x_new, got.x_new, rtol=0, atol=1e-12)
    assert force.moving_mask(wl.tag, wl.move_mask).sum() > 3000
