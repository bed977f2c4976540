"""Pins of the CPU oracle against mathematics and the paper, independent of the oracle's own code.

Each test checks the oracle against something it does not compute itself: a
value printed in the paper, an integral, a finite difference, a symmetry of
the exact problem, an analytic special case, or an independent search method.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

import synth
from synth import meshes as M
from oracle import cells, force, geometry, hvp, kernel, metrics, neighbors, step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- kernel (Eq. 16-17)

def test_kernel_2d_normalised_by_paper_constant():
    """Eq. 17 prints alpha_2 = 7/(4 pi h^2): with it the Eq. 16 polynomial must
    integrate to one over the plane. Pins the polynomial against the paper."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    for h in (0.3, 1.0, 2.7):
        val, _ = integrate.quad(lambda r: 2 * math.pi * r * kernel.W(r, h, d=2), 0, 2 * h)
        assert abs(val - 1.0) < 1e-12
        assert abs(kernel.alpha(h, 2) * h * h - g["alpha_2d_coeff_value"]) < 1e-15


def test_kernel_3d_normalised_and_printed_constant_is_not():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    for h in (0.013, 0.5, 1.7):
        val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * kernel.W(r, h), 0, 2 * h)
        assert abs(val - 1.0) < 1e-12
    # with the printed 3-D coefficient the integral is 16/6, not 1 (garbled Eq. 17)
    printed = g["alpha_3d_coeff_printed_value"]
    h = 1.0
    val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * kernel.W(r, h) / kernel.alpha(h) * printed, 0, 2)
    assert abs(val - 16.0 / 6.0) < 1e-12


def test_kernel_support_and_values():
    h = 0.7
    assert kernel.W(2 * h, h) == 0.0 and kernel.W(3 * h, h) == 0.0
    assert abs(kernel.W(0.0, h) - kernel.alpha(h)) < 1e-15       # (1)^4 (1) at q = 0


def test_dW_dr_matches_central_difference():
    h = 0.37
    r = np.linspace(0.01, 2 * h - 0.01, 57)
    eps = 1e-6
    fd = (kernel.W(r + eps, h) - kernel.W(r - eps, h)) / (2 * eps)
    assert np.allclose(kernel.dW_dr(r, h), fd, rtol=1e-7, atol=1e-9 * kernel.alpha(h) / h)


def test_two_particle_force_is_minus_kernel_gradient():
    """Eq. 15 with prefactor 1: a_0 = -dW/dr e_01, equal and opposite, zero beyond 2h."""
    mesh = M.cube()
    dx = 0.05
    h = synth.f32(1.3 * dx)
    for dist in (0.3 * h, 1.0 * h, 1.9 * h, 2.05 * h):
        p = np.array([[0.5, 0.5, 0.5], [0.5 + dist, 0.5, 0.5]], np.float32)
        wl = synth.workload.custom_workload(mesh, dx, p, [3, 3], move_mask=1 << 3)
        a, S, cnt = force.accel(wl)
        r = float(p[1, 0]) - float(p[0, 0])
        eps = 1e-7
        dWdr = (kernel.W(r + eps, h) - kernel.W(r - eps, h)) / (2 * eps)
        if r < 2 * h:
            assert cnt.tolist() == [1, 1]
            assert abs(a[0, 0] - dWdr) <= 1e-6 * abs(dWdr)     # -dW/dr * e_01, e_01 = -x
            assert abs(a[0, 1]) == 0 and abs(a[0, 2]) == 0
            assert np.array_equal(a[0], -a[1])
        else:
            assert cnt.tolist() == [0, 0] and not a.any()


# --------------------------------------------------------------------------- neighbours

def _cloud(n, seed, dx=0.05, box=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0, box, (n, 3))


def test_neighbors_equal_kdtree_search():
    """Brute-force pair enumeration = k-d tree ball search filtered by the same
    binary32 predicate; includes adversarial pairs within an ulp of r_c."""
    dx = 0.05
    h = synth.f32(1.3 * dx)
    rc = np.float32(2) * np.float32(h)
    p = _cloud(2500, 7, dx, box=0.6)
    rng = np.random.Generator(np.random.PCG64(8))
    extra = []
    for _ in range(200):                  # pairs at exactly r_c and 1 ulp on either side
        a = rng.uniform(0.1, 0.5, 3).astype(np.float32)
        for off in (np.nextafter(rc, np.float32(0)), rc, np.nextafter(rc, np.float32(1))):
            b = a.copy()
            b[rng.integers(3)] += np.float32(off)
            extra += [a, b]
    p = np.concatenate([p.astype(np.float32), np.array(extra, np.float32)], 0)
    mesh = M.cube((0, 0, 0), (1, 1, 1))
    wl = synth.workload.custom_workload(mesh, dx, p, np.full(len(p), 3))
    nb = neighbors.neighbor_lists(wl, pos32=wl.pos)
    tree = cKDTree(wl.pos.astype(np.float64))
    rc2 = neighbors.rc2_f32(h)
    for i in range(wl.n):
        cand = np.array(sorted(j for j in tree.query_ball_point(wl.pos[i].astype(np.float64),
                                                                float(rc) * (1 + 1e-5)) if j != i))
        if len(cand):
            d = (wl.pos[i] - wl.pos[cand]).astype(np.float32)
            d2 = np.float32(np.float32(d[:, 0] * d[:, 0]) + np.float32(d[:, 1] * d[:, 1])) \
                + np.float32(d[:, 2] * d[:, 2])
            cand = cand[d2.astype(np.float32) < rc2]
        assert np.array_equal(nb[i], cand), i


def test_neighbor_predicate_is_strict_at_rc():
    """Two particles exactly r_c apart along an axis are not neighbours, one
    ulp closer they are (q < 2 strictly inside the support)."""
    dx = 0.05
    h = synth.f32(1.3 * dx)
    rc = np.float32(2) * np.float32(h)
    a = np.float32(0.0)
    for off, want in ((rc, 0), (np.nextafter(rc, np.float32(0)), 1)):
        p = np.array([[a, 0.5, 0.5], [a + off, 0.5, 0.5]], np.float32)
        assert float(p[1, 0]) - float(p[0, 0]) == float(off)
        wl = synth.workload.custom_workload(M.cube(), dx, p, [3, 3])
        nb = neighbors.neighbor_lists(wl)
        assert len(nb[0]) == want


# --------------------------------------------------------------------------- cell list

def test_cell_keys_contain_particles_and_order_is_key_then_id():
    wl = synth.cube_workload(n=8, seed=3)
    geo = wl.geoms[0]
    pos = wl.pos.copy()
    pos[:5] = [[-5, 0.5, 0.5], [0.5, 9, 0.5], [np.nan, 0.5, 0.5], [0.5, 0.5, -1e30], [2, 2, 2]]
    keys = cells.cell_keys(wl, pos32=pos)
    # the grid's cells halved along x: edges (cell / 2, cell, cell)
    cell = 1.0 / np.float64(geo.inv_cell) * np.array([0.5, 1.0, 1.0])
    nx, ny, nz = 2 * int(geo.dims[0]), int(geo.dims[1]), int(geo.dims[2])
    assert cells.total_cells(wl) == nx * ny * nz
    fin = np.all(np.isfinite(pos), 1)
    c = np.stack([keys % nx, (keys // nx) % ny, keys // (nx * ny)], 1)
    assert (c[fin] >= 0).all() and (c[fin] < [nx, ny, nz]).all()
    inside = np.all(np.isfinite(pos), 1) & np.all(pos > -1, 1) & np.all(pos < 1.5, 1)
    lo = geo.origin.astype(np.float64) + c * cell
    x = pos.astype(np.float64)
    tol = 1e-5 * cell
    assert np.all(x[inside] >= lo[inside] - tol) and np.all(x[inside] < lo[inside] + cell + tol)
    # both halves of the grid's cells are used
    assert np.any(c[inside, 0] % 2 == 0) and np.any(c[inside, 0] % 2 == 1)
    assert keys[0] == (int(c[0, 2]) * ny + int(c[0, 1])) * nx + 0            # clamped low in x
    assert c[1, 1] == ny - 1 and c[3, 2] == 0                                 # clamped
    assert keys[2] == cells.total_cells(wl)                                   # NaN: quarantine key
    order = cells.sort_order(keys, wl.ids)
    want = [i for _, i in sorted(zip(keys.tolist(), wl.ids.tolist()))]
    assert order.tolist() == want
    cs = cells.cell_start(keys[order], cells.total_cells(wl))
    counts = {}
    for k in keys.tolist():
        counts[k] = counts.get(k, 0) + 1
    for k in range(cells.total_cells(wl) + 1):
        assert cs[k + 1] - cs[k] == counts.get(k, 0)
    assert cs[-1] == wl.n and len(cs) == cells.total_cells(wl) + 2


@pytest.mark.parametrize("dims,slab", [((7, 10, 5), 3), ((7, 10, 5), 4), ((4, 9, 3), 1), ((5, 6, 2), 6)])
def test_slab_keys_enumerate_the_cells_with_contiguous_x_rows(dims, slab):
    """The slab key is a bijection of the cells onto [0, ncell), x rows are
    runs of consecutive keys, the rows of one slab and plane are consecutive,
    and a single slab is the plain x-fastest index."""
    nx, ny, nz = dims
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    k = cells.linear_key(g, dims, slab)
    assert sorted(k.tolist()) == list(range(nx * ny * nz))
    right = g[:, 0] + 1 < nx
    kr = cells.linear_key(g[right] + [1, 0, 0], dims, slab)
    assert np.array_equal(kr, k[right] + 1)
    # walking the keys in order: slab index never decreases, z within a slab never decreases
    inv = np.empty_like(k)
    inv[k] = np.arange(len(k))
    c = g[inv]
    s = c[:, 1] // slab
    assert np.all(np.diff(s) >= 0)
    same = np.diff(s) == 0
    assert np.all(np.diff(c[:, 2])[same] >= 0)
    plain = (g[:, 2] * ny + g[:, 1]) * nx + g[:, 0]
    assert np.array_equal(cells.linear_key(g, dims, 0), plain)
    assert np.array_equal(cells.linear_key(g, dims, ny), plain)


# --------------------------------------------------------------------------- forces

def test_dyadic_lattice_interior_force_vanishes():
    wl = synth.dyadic_lattice_workload(m=14)
    h = wl.geoms[0].h
    x = wl.pos.astype(np.float64)
    lo, hi = x.min(0), x.max(0)
    interior = np.all((x - lo >= 2 * h) & (hi - x >= 2 * h), 1)
    rec = np.nonzero(interior)[0]
    assert len(rec) > 20
    a, S, cnt = force.accel(wl, rec)
    assert (np.linalg.norm(a, axis=1) <= 1e-14 * S).all()
    assert (cnt == cnt[0]).all()
    # lattice points strictly inside radius 2.6 dx: 80 neighbours (Gauss circle count in 3-D)
    ks = np.arange(-3, 4)
    g = np.stack(np.meshgrid(ks, ks, ks, indexing="ij"), -1).reshape(-1, 3)
    r = np.linalg.norm(g, axis=1)
    assert cnt[0] == int(np.sum((r > 0) & (r * wl.geoms[0].dx < 2 * h)))


def test_momentum_and_angular_momentum_conserved_for_mutual_forces():
    """All particles in one class, none fixed: forces are pairwise equal and
    opposite and central, so sum a = 0 and sum x x a = 0."""
    rng = np.random.Generator(np.random.PCG64(11))
    dx = 0.05
    p = (np.stack(np.meshgrid(*[np.arange(10) * dx] * 3, indexing="ij"), -1).reshape(-1, 3)
         + 0.2 + rng.uniform(-0.3, 0.3, (1000, 3)) * dx)
    wl = synth.workload.custom_workload(M.cube(), dx, p, np.full(len(p), 3), move_mask=1 << 3)
    a, S, _ = force.accel(wl)
    x = wl.pos.astype(np.float64)
    assert np.linalg.norm(a.sum(0)) <= 1e-12 * S.sum()
    assert np.linalg.norm(np.cross(x, a).sum(0)) <= 1e-12 * S.sum()


def test_class_interaction_rule():
    """A surface particle is not pushed by a volume particle; the volume
    particle is pushed by the surface particle (section 2.2 / 3.3.4)."""
    dx = 0.05
    p = np.array([[0.5, 0.5, 1.0], [0.5, 0.5, 1.0 - 0.8 * dx]], np.float32)
    wl = synth.workload.custom_workload(M.cube(), dx, p, [2, 3], owner=[0, -1])
    a, S, cnt = force.accel(wl)
    assert cnt.tolist() == [0, 1] and not a[0].any() and a[1, 2] < 0


def test_step_moves_fastest_particle_exactly_h_over_16():
    """Time-step reading: the particle with the largest acceleration moves h/16."""
    rng = np.random.Generator(np.random.PCG64(12))
    dx = 0.05
    p = np.stack(np.meshgrid(*[np.arange(8) * dx] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.3
    p = p + rng.uniform(-0.3, 0.3, p.shape) * dx
    wl = synth.workload.custom_workload(M.cube(), dx, p, np.full(len(p), 3), move_mask=1 << 3)
    out = step.relax_step(wl)
    dr = np.linalg.norm(out.dr, axis=1)
    i = int(np.argmax(np.linalg.norm(out.a, axis=1)))
    assert abs(dr[i] - wl.geoms[0].h / 16) <= 1e-13 * wl.geoms[0].h
    assert dr.max() <= wl.geoms[0].h / 16 * (1 + 1e-13)


# --------------------------------------------------------------------------- projection

def _cube_face_owner(mesh, p, axis, side):
    """Owner facet of a point on a cube face by the paper's cross-product test (Fig. 8)."""
    for t, (i, j, k) in enumerate(mesh.tri):
        A, B, C = mesh.vert[i], mesh.vert[j], mesh.vert[k]
        if not (A[axis] == side and B[axis] == side and C[axis] == side):
            continue
        n = np.cross(B - A, C - A)
        s = [np.dot(np.cross(Q - P, p - P), n) for P, Q in ((A, B), (B, C), (C, A))]
        if min(s) >= 0:
            return t
    return -1


def test_surface_projection_cube_closed_form():
    """On a cube face the projection of an off-plane point is exact: the normal
    coordinate becomes the face coordinate, the tangential ones are unchanged,
    and the owner is the facet that contains the point."""
    mesh = M.cube()
    wl = synth.workload.custom_workload(mesh, 0.05, np.zeros((1, 3)), [2], owner=[0])
    rng = np.random.Generator(np.random.PCG64(13))
    R = wl.geoms[0].proj_radius
    for axis in range(3):
        for side in (0.0, 1.0):
            y = rng.uniform(0.1, 0.9, (40, 3))
            off = rng.uniform(-0.5, 0.5, 40) * R
            y[:, axis] = side + off
            ok, foot, own, mg = step.project_surface(wl, y, 0)
            assert ok.all()
            want = y.copy()
            want[:, axis] = side
            assert np.array_equal(foot, want)
            for q in range(40):
                assert own[q] == _cube_face_owner(mesh, want[q], axis, side)


def test_surface_projection_reverts_beyond_radius():
    mesh = M.cube()
    wl = synth.workload.custom_workload(mesh, 0.05, np.zeros((1, 3)), [2], owner=[0])
    R = wl.geoms[0].proj_radius
    y = np.array([[1.0 + 2 * R, 0.5, 1.0 + 2 * R], [0.5, 0.5, 1.0 + 1.5 * R]])
    ok, foot, own, mg = step.project_surface(wl, y, 0)
    assert not ok.any() and (own == -1).all()


def test_surface_step_on_cube_keeps_particles_on_faces():
    wl = synth.cube_workload(n=8, seed=4)
    out = step.relax_step(wl)
    s = wl.tag == 2
    x = out.pos32[s].astype(np.float64)
    # every surface particle has one coordinate exactly 0 or 1 (its face)
    on_face = np.any((x == 0.0) | (x == 1.0), axis=1)
    assert on_face.all()
    assert (np.abs(out.x_new[s] - wl.pos[s]).max() > 0)
    # Eq. 25 on a face: the in-face coordinates move by tau*a, the normal one not at all
    x0 = wl.pos.astype(np.float64)
    moved = 0
    for i in np.nonzero(s & ~out.reverted)[0]:
        axis = int(np.nonzero((x0[i] == 0.0) | (x0[i] == 1.0))[0][0])
        want = x0[i] + out.tau[0] * out.a[i]
        want[axis] = x0[i, axis]
        if np.all((want > 0) & (want < 1) | (np.arange(3) == axis)):
            assert np.allclose(out.x_new[i], want, rtol=0, atol=1e-15)
            assert out.dr[i, axis] == 0.0
            moved += 1
    assert moved > 100


def test_icosphere_projection_lies_on_facets():
    wl = synth.sphere_workload(level=2, dx=0.12, seed=6)
    out = step.relax_step(wl)
    s = (wl.tag == 2) & ~out.reverted
    A, B, C, n = geometry.facet_frames(wl.geoms[0].mesh.vert, wl.geoms[0].mesh.tri)
    p = out.x_new[s]
    o = out.owner[s]
    d = np.einsum("ij,ij->i", p - A[o], n[o])
    assert np.abs(d).max() <= 1e-6 * wl.geoms[0].dx
    la, lb, lc = geometry.barycentric(p, A[o], B[o], C[o])
    assert np.minimum(np.minimum(la, lb), lc).min() >= -1e-12


# --------------------------------------------------------------------------- feature lines

def test_feature_particle_on_straight_edge_moves_by_tangential_component():
    wl = synth.cube_workload(n=8, seed=5, with_volume=False, with_surface=False,
                             move_mask=1 << synth.FEATURE)
    out = step.relax_step(wl)
    f = np.nonzero(wl.tag == 1)[0]
    segs = step.batch_segments(wl)
    moved = 0
    for i in f:
        slot = wl.owner[i]
        s = wl.feat_seg[slot]
        P0, t = segs[0][s], segs[3][s]
        want_u = wl.feat_u[slot] + float(np.dot(out.a[i] * out.tau[0], t))
        if out.reverted[i]:
            assert want_u < 0 or want_u > segs[2][s]
            continue
        assert abs(out.feat_u[slot] - want_u) <= 1e-15
        assert np.allclose(out.x_new[i], P0 + want_u * t, atol=1e-15)
        moved += 1
    assert moved > 0


def test_feature_walk_on_closed_loop_wraps():
    square = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 0]], np.float64)
    lines = M.FeatureLines.from_polylines([square], [1])
    segs = (lines.seg_p[:, 0], lines.seg_p[:, 1], np.ones(4), None,
            np.zeros(4, int), np.full(4, 4), np.ones(4, int))
    ok, s, u, _ = step.advance_feature(3, 0.9, 0.3, segs)
    assert ok and s == 0 and abs(u - 0.2) < 1e-15
    ok, s, u, _ = step.advance_feature(0, 0.1, -0.35, segs)
    assert ok and s == 3 and abs(u - 0.75) < 1e-15
    ok, s, u, _ = step.advance_feature(2, 0.1, -0.35, segs)
    assert ok and s == 1 and abs(u - 0.75) < 1e-15
    ok, s, u, _ = step.advance_feature(1, 0.5, 2.25, segs)      # crosses two segments
    assert ok and s == 3 and abs(u - 0.75) < 1e-15
    open_segs = segs[:6] + (np.zeros(4, int),)
    ok, s, u, _ = step.advance_feature(3, 0.9, 0.3, open_segs)
    assert not ok and s == 3 and u == 0.9


# --------------------------------------------------------------------------- signed distance

def test_signed_distance_matches_analytic_box():
    lo, hi = np.array([0.1, -0.2, 0.3]), np.array([0.9, 0.5, 1.2])
    mesh = M.cube(lo, hi)
    rng = np.random.Generator(np.random.PCG64(14))
    p = rng.uniform(lo - 0.4, hi + 0.4, (400, 3))
    q = np.abs(p - (lo + hi) / 2) - (hi - lo) / 2
    want = np.linalg.norm(np.maximum(q, 0), axis=1) + np.minimum(q.max(1), 0)
    got = geometry.signed_distance_many(p, mesh.vert, mesh.tri)
    assert np.allclose(got, want, atol=1e-13)
    got1 = geometry.signed_distance(p[:30], mesh.vert, mesh.tri)
    assert np.allclose(got1, want[:30], atol=1e-13)


def test_signed_distance_sphere_within_facet_sag():
    mesh = M.icosphere(3)
    rng = np.random.Generator(np.random.PCG64(15))
    p = rng.normal(size=(300, 3))
    p *= (rng.uniform(0.5, 1.5, 300) / np.linalg.norm(p, axis=1))[:, None]
    A, B, C, n = geometry.facet_frames(mesh.vert, mesh.tri)
    sag = 1.0 - np.min(np.einsum("ij,ij->i", n, A))
    sd = geometry.signed_distance_many(p, mesh.vert, mesh.tri)
    assert np.all(np.abs(sd - (np.linalg.norm(p, axis=1) - 1.0)) <= sag + 1e-12)


def test_volume_particle_pushed_outside_reverts():
    """A volume particle next to a face with a strong push outward returns."""
    dx = 0.05
    p = np.array([[0.5, 0.5, 0.999], [0.5, 0.5, 0.999 - 0.5 * dx]], np.float32)
    wl = synth.workload.custom_workload(M.cube(), dx, p, [3, 4], move_mask=1 << 3)
    out = step.relax_step(wl)
    assert out.reverted[0] and np.array_equal(out.pos32[0], wl.pos[0])


# --------------------------------------------------------------------------- Jacobian

def _small_volume_case(seed=16, fixed_frac=0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = 0.05
    p = np.stack(np.meshgrid(*[np.arange(7) * dx] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.3
    p = p + rng.uniform(-0.3, 0.3, p.shape) * dx
    tag = np.where(rng.uniform(size=len(p)) < fixed_frac, 4, 3)
    return synth.workload.custom_workload(M.cube(), dx, p, tag, move_mask=1 << 3)


def test_jvp_matches_central_difference_of_force():
    wl = _small_volume_case(fixed_frac=0.2)
    rng = np.random.Generator(np.random.PCG64(17))
    v = rng.normal(size=(wl.n, 3))
    v[wl.tag == 4] = 0
    x = wl.pos.astype(np.float64)
    eps = 1e-6 * wl.geoms[0].dx
    ap, _, _ = force.accel(wl, pos64=x + eps * v)
    am, _, _ = force.accel(wl, pos64=x - eps * v)
    fd = (ap - am) / (2 * eps)
    jv = hvp.jvp(wl, v)
    assert np.linalg.norm(jv - fd) <= 1e-6 * np.linalg.norm(fd)


def test_jacobian_symmetric_and_translation_null_space():
    wl = _small_volume_case(fixed_frac=0.2)
    rng = np.random.Generator(np.random.PCG64(18))
    u, v = rng.normal(size=(2, wl.n, 3))
    u[wl.tag == 4] = 0
    v[wl.tag == 4] = 0
    assert abs(np.sum(u * hvp.jvp(wl, v)) - np.sum(v * hvp.jvp(wl, u))) <= 1e-10 * np.abs(
        np.sum(u * hvp.jvp(wl, v)))
    assert abs(np.sum(u * hvp.jvp(wl, v)) - np.sum(v * hvp.vjp(wl, u))) <= 1e-10 * np.abs(
        np.sum(u * hvp.jvp(wl, v)))
    free = _small_volume_case(fixed_frac=0.0)
    e = np.tile([0.3, -1.0, 0.5], (free.n, 1))
    ref = np.linalg.norm(hvp.jvp(free, rng.normal(size=(free.n, 3))))
    assert np.linalg.norm(hvp.jvp(free, e)) <= 1e-12 * ref


def test_force_is_minus_energy_gradient():
    wl = _small_volume_case(fixed_frac=0.2)
    rng = np.random.Generator(np.random.PCG64(19))
    v = rng.normal(size=(wl.n, 3))
    v[wl.tag == 4] = 0
    x = wl.pos.astype(np.float64)
    eps = 1e-7 * wl.geoms[0].dx
    dE = (hvp.energy(wl, x + eps * v) - hvp.energy(wl, x - eps * v)) / (2 * eps)
    a, _, _ = force.accel(wl)
    assert abs(dE + np.sum(a * v)) <= 1e-6 * abs(dE)


def test_vjp_is_transpose_with_several_moving_ranks():
    wl = synth.cube_workload(n=6, seed=20)
    rng = np.random.Generator(np.random.PCG64(21))
    u, v = rng.normal(size=(2, wl.n, 3))
    lhs = np.sum(u * hvp.jvp(wl, v))
    rhs = np.sum(v * hvp.vjp(wl, u))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


# --------------------------------------------------------------------------- metrics

def test_lattice_density_equals_interior_kernel_sum():
    wl = synth.dyadic_lattice_workload(m=12)
    dx, h = wl.geoms[0].dx, wl.geoms[0].h
    rho0 = metrics.lattice_density(dx, float(h))
    rho = metrics.densities(wl)
    x = wl.pos.astype(np.float64)
    interior = np.all((x - x.min(0) >= 2 * h) & (x.max(0) - x >= 2 * h), 1)
    assert np.allclose(rho[interior], rho0, rtol=1e-13)
    # a perfect lattice has (numerically) zero uniformity loss at interior particles
    assert np.max(np.abs(rho[interior] / rho0 - 1)) < 1e-13


def _cube_facet_on(mesh, axis, value):
    """Index of a facet of the axis-aligned cube whose three vertices lie on the plane x[axis] = value."""
    v = mesh.vert[mesh.tri]
    return int(np.nonzero(np.all(v[:, :, axis] == value, axis=1))[0][0])


def _cube_segment_along(mesh, axis):
    """Index of a feature segment of the cube whose end points differ only along `axis`."""
    p = mesh.lines.seg_p
    d = p[:, 1] - p[:, 0]
    other = [a for a in range(3) if a != axis]
    return int(np.nonzero((np.abs(d[:, axis]) > 0) & np.all(d[:, other] == 0, axis=1))[0][0])


def test_residual_closed_form_on_cube_face_edge_and_volume():
    """R = sqrt(mean over moving particles of |P a|^2) with P = I - n n^T on a
    cube face (n = +z: the z part of a drops), P = t t^T on a straight edge
    (t = x: only the x part stays), I for a volume particle; a fixed particle is
    not in the mean. The expected value is written from the cube's geometry."""
    mesh = M.cube()
    dx = 1.0 / 8
    top = _cube_facet_on(mesh, 2, 1.0)
    seg = _cube_segment_along(mesh, 0)
    p0 = mesh.lines.seg_p[seg, 0]
    pos = np.array([[0.4, 0.6, 1.0], p0 + [0.3 * np.sign(mesh.lines.seg_p[seg, 1, 0] - p0[0]), 0, 0],
                    [0.5, 0.5, 0.5], [0.25, 0.25, 0.25]])
    wl = synth.workload.custom_workload(mesh, dx, pos, [2, 1, 3, 4], owner=[top, 0, -1, -1],
                                        feat_seg=[seg], feat_u=[0.3])
    a = np.array([[3.0, -4.0, 7.0], [2.0, 5.0, -6.0], [1.0, -2.0, 2.0], [9.0, 9.0, 9.0]])
    pa = metrics.projected_accel(wl, a, wl.owner, wl.feat_seg)
    assert np.allclose(pa[0], [3.0, -4.0, 0.0], atol=1e-15)
    assert np.allclose(pa[1], [2.0, 0.0, 0.0], atol=1e-15)
    assert np.array_equal(pa[2], a[2])
    want = math.sqrt((25.0 + 4.0 + 9.0) / 3.0)
    assert metrics.residual(wl, a, wl.owner, wl.feat_seg) == pytest.approx(want, rel=1e-15)
    # only the moving classes count: with the surface class fixed the mean runs over two particles
    wl.move_mask = (1 << 1) | (1 << 3)
    assert metrics.residual(wl, a, wl.owner, wl.feat_seg) == pytest.approx(math.sqrt((4.0 + 9.0) / 2.0), rel=1e-15)


def test_residual_vanishes_on_exact_lattice_interior():
    """On the exact dyadic lattice with the particles within 2h of the edge of
    the block fixed, every moving particle has zero force: R = 0 up to rounding
    of the force sums (1e-14 of the one-sided force scale)."""
    wl = synth.dyadic_lattice_workload(m=12)
    h = float(wl.geoms[0].h)
    x = wl.pos.astype(np.float64)
    interior = np.all((x - x.min(0) >= 2 * h) & (x.max(0) - x >= 2 * h), 1)
    wl.tag = np.where(interior, 3, 4).astype(np.int32)
    a, S, _ = force.accel(wl)
    R = metrics.residual(wl, a, wl.owner, wl.feat_seg)
    assert interior.sum() > 50
    assert R <= 1e-14 * float(np.max(S[interior]))
    # and the same lattice with one interior particle displaced has R > 0
    k = int(np.nonzero(interior)[0][len(np.nonzero(interior)[0]) // 2])
    wl.pos = wl.pos.copy()
    wl.pos[k, 0] += np.float32(wl.geoms[0].dx / 8)
    a, S, _ = force.accel(wl)
    assert metrics.residual(wl, a, wl.owner, wl.feat_seg) > 1e-3 * float(np.max(S[interior]))


def test_uniformity_loss_closed_form_with_displaced_particles():
    """Nearest-neighbour support (2h = 1.2 dx): in an exact cubic lattice every
    particle has 6 neighbours at dx, so rho0 = W(0) + 6 W(dx). A particle moved
    by d along x has two neighbours at dx -+ d and four at sqrt(dx^2 + d^2);
    one moved along y the same. Two such movers far apart, every other particle
    fixed: L = mean over the two of (rho/rho0 - 1)^2."""
    dx = 2.0 ** -5
    m = 12
    c = (np.arange(m) + 0.5) * dx
    pos = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    idx = lambda i, j, k: (i * m + j) * m + k
    a, b = idx(3, 3, 3), idx(8, 8, 8)
    d1, d2 = dx / 8, dx / 4
    pos[a, 0] += d1
    pos[b, 1] -= d2
    tag = np.full(len(pos), 4, np.int32)
    tag[[a, b]] = 3
    wl = synth.workload.custom_workload(M.cube((0, 0, 0), (m * dx,) * 3), dx, pos.astype(np.float32), tag,
                                        move_mask=1 << 3)
    h = 0.6 * dx
    wl.geoms[0].h = h
    W = lambda r: kernel.W(np.asarray(r, np.float64), h)
    rho0 = W(0.0) + 6 * W(dx)
    assert metrics.lattice_density(dx, h) == pytest.approx(rho0, rel=1e-15)
    rho = lambda d: W(0.0) + W(dx - d) + W(dx + d) + 4 * W(math.hypot(dx, d))
    want = 0.5 * ((rho(d1) / rho0 - 1) ** 2 + (rho(d2) / rho0 - 1) ** 2)
    assert want > 0
    assert metrics.uniformity_loss(wl) == pytest.approx(want, rel=1e-12)
    # the undisplaced lattice has zero loss
    wl0 = synth.workload.custom_workload(M.cube((0, 0, 0), (m * dx,) * 3), dx,
                                         np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3), tag,
                                         move_mask=1 << 3)
    wl0.geoms[0].h = h
    assert metrics.uniformity_loss(wl0) <= 1e-28
