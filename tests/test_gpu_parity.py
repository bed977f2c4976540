"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Bars (the tolerances the method's hot path is held to):
  * cell order, cell_start and neighbour sets: bit-exact
  * forces: |a_gpu - a_64| <= 1e-5 * S_i  with S_i = sum_j K (1-q/2)^3 |r_ij|
  * positions after one step: |x_gpu - x_64|_inf <= 1e-5 * max(|x_64|_inf, dx)
    for particles whose projection/revert decision is not within rounding of
    flipping (the oracle flags those as margin; they must still satisfy the
    geometric invariants)
Every comparison starts from the same binary32 state.
"""
import numpy as np
import pytest

import synth
from oracle import cells as ocells
from oracle import force as oforce
from oracle import geometry as ogeo
from oracle import hvp as ohvp
from oracle import neighbors as onb
from oracle import step as ostep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _relaxer(wl):
    from paper_2501_03056_amd import Relaxer
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Relaxer(wl, device=0)


def _slab(wl, S):
    """The same workload with its cell keys cut into slabs of S cell rows."""
    for g in wl.geoms:
        g.slab = S
    return wl


CASES = {
    "cube_n8": lambda: synth.cube_workload(n=8, seed=1),
    "sphere_l3_slab3": lambda: _slab(synth.sphere_workload(level=3, dx=0.08, seed=2), 3),
    "cube_n10_k1_slab4": lambda: _slab(synth.cube_workload(n=10, seed=7, k=1), 4),
    "tetra_slab5": lambda: _slab(synth.tetra_workload(dx=0.06, seed=5), 5),
    "cube_n24": lambda: synth.cube_workload(n=24, seed=1),
    "cube_n10_k1": lambda: synth.cube_workload(n=10, seed=7, k=1),
    "sphere_l3": lambda: synth.sphere_workload(level=3, dx=0.08, seed=2),
    "tetra": lambda: synth.tetra_workload(dx=0.06, seed=5),
}


@pytest.mark.parametrize("case", ["cube_n8", "sphere_l3", "cube_n10_k1", "sphere_l3_slab3", "cube_n10_k1_slab4"])
def test_cells_bit_exact(case):
    wl = CASES[case]()
    r = _relaxer(wl)
    r.build_cells()
    torch.cuda.synchronize()
    keys = ocells.cell_keys(wl)
    order = ocells.sort_order(keys, wl.ids)
    cs = ocells.cell_start(keys[order], ocells.total_cells(wl))
    assert np.array_equal(r.id.cpu().numpy(), order)
    assert np.array_equal(r.cell_start.cpu().numpy(), cs)
    pos = r.pos.cpu().numpy()
    assert np.array_equal(pos[:, :3], wl.pos[order])
    assert np.array_equal(r.owner.cpu().numpy(), wl.owner[order])
    # a second rebuild of an already sorted state is the identity
    before = r.pos.clone()
    r.build_cells()
    assert torch.equal(before, r.pos)


@pytest.mark.parametrize("case", ["cube_n8", "sphere_l3", "cube_n10_k1", "sphere_l3_slab3", "cube_n10_k1_slab4"])
def test_neighbor_sets_bit_exact(case):
    wl = CASES[case]()
    r = _relaxer(wl)
    r.build_cells()
    count, lst = r.neighbors(cap=200)
    count = count.cpu().numpy()
    lst = lst.cpu().numpy()
    ids = r.id.cpu().numpy()
    ref = onb.neighbor_lists(wl)
    for s in range(wl.n):
        i = ids[s]
        got = np.sort(ids[lst[s, : count[s]]])
        assert count[s] == len(ref[i]) and np.array_equal(got, ref[i]), (s, i)


def test_neighbor_sets_adversarial_pairs_at_cell_faces():
    """Pairs within an ulp of r_c, straddling particle-cell faces."""
    dx = 0.05
    h = synth.f32(1.3 * dx)
    rc = np.float32(2) * np.float32(h)
    from synth import meshes as M
    geo_wl = synth.workload.custom_workload(M.cube(), dx, np.zeros((1, 3)), [3])
    g = geo_wl.geoms[0]
    cell = np.float32(1) / np.float32(g.inv_cell)
    rng = np.random.Generator(np.random.PCG64(31))
    pts = []
    for _ in range(300):
        c = rng.integers(3, 10, 3)
        a = (g.origin + c.astype(np.float32) * cell).astype(np.float32)    # on a cell corner
        a = np.nextafter(a, a + np.float32(rng.choice([-1, 1])))
        for off in (np.nextafter(rc, np.float32(0)), rc):
            b = a.copy()
            ax = rng.integers(3)
            b[ax] = np.float32(a[ax] + off)
            pts += [a, b]
        # random directions at just under / at the support radius: the stencil
        # corners, where the row and x-range culling is tightest
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        for scale in (1 - 3e-7, 1 - 1e-7, 1.0):
            pts += [a, (a + u * float(rc) * scale).astype(np.float32)]
    p = np.array(pts, np.float32)
    wl = synth.workload.custom_workload(M.cube(), dx, p, np.full(len(p), 3))
    r = _relaxer(wl)
    r.build_cells()
    count, lst = r.neighbors(cap=1024)
    count, lst, ids = count.cpu().numpy(), lst.cpu().numpy(), r.id.cpu().numpy()
    assert count.max() < 1024
    ref = onb.neighbor_lists(wl)
    for s in range(wl.n):
        assert count[s] == len(ref[ids[s]])
        assert np.array_equal(np.sort(ids[lst[s, : count[s]]]), ref[ids[s]])


@pytest.mark.parametrize("case", ["cube_n24", "sphere_l3", "tetra", "cube_n10_k1", "sphere_l3_slab3",
                                  "tetra_slab5"])
def test_forces_within_1e5_of_fp64(case):
    wl = CASES[case]()
    r = _relaxer(wl)
    r.build_cells()
    r.relax_step(count_pairs=True)
    acc = r.by_id(r.accel)
    a64, S, cnt = oforce.accel(wl)
    mov = oforce.moving_mask(wl.tag, wl.move_mask)
    err = np.linalg.norm(acc[:, :3].astype(np.float64) - a64, axis=1)
    assert np.all(err[mov] <= 1e-5 * S[mov]), float(np.max(err[mov] / np.maximum(S[mov], 1e-300)))
    assert np.array_equal(acc[:, 3].astype(np.int64), np.where(mov, cnt, 0))
    assert not acc[~mov, :3].any()
    amax = oforce.amax_per_geometry(wl, a64)
    assert np.allclose(r.amax.cpu().numpy(), amax, rtol=1e-5)
    assert r.read_status() == 0


def _compare_step(wl, r, ref, check_owner=True):
    pos, owner, fs, fu = r.host_state()
    ok = ~ref.margin
    x = ref.pos32.astype(np.float64)
    dx = wl.geoms[0].dx
    tol = 1e-5 * np.maximum(np.abs(x).max(1), dx)
    err = np.abs(pos.astype(np.float64) - x).max(1)
    bad = ok & (err > tol)
    assert not bad.any(), (int(bad.sum()), np.nonzero(bad)[0][:10], float(err[ok].max()))
    if check_owner:
        s = ok & (wl.tag == synth.SURFACE)
        assert np.array_equal(owner[s], ref.owner[s])
    f = np.nonzero(ok & (wl.tag == synth.FEATURE))[0]
    if len(f):
        slots = wl.owner[f]
        assert np.array_equal(fs[slots], ref.feat_seg[slots])
        assert np.allclose(fu[slots], ref.feat_u[slots], rtol=0, atol=1e-5 * dx)
    return pos, owner


@pytest.mark.parametrize("case", ["cube_n24", "sphere_l3", "tetra", "cube_n10_k1", "sphere_l3_slab3",
                                  "tetra_slab5"])
def test_one_step_positions_within_1e5_of_fp64(case):
    wl = CASES[case]()
    r = _relaxer(wl)
    r.step()
    ref = ostep.relax_step(wl)
    _compare_step(wl, r, ref)
    c = r.counters.cpu().numpy()
    s = wl.tag == synth.SURFACE
    assert abs(int(c[0]) - int(np.sum(ref.reverted & s))) <= int(np.sum(ref.margin & s))
    assert r.read_status() == 0


GEAR_TIERS = {"feature": (0.04, 1 << synth.FEATURE), "surface": (0.04, 1 << synth.SURFACE),
              "volume": (0.06, 1 << synth.VOLUME)}


@pytest.mark.parametrize("tier", list(GEAR_TIERS))
def test_gear_tier_forces_and_one_step_match_oracle(tier):
    """The gear (coarse 288-sample outline, 5,760 facets) relaxed tier by tier:
    forces and one step of the moving class against the oracle."""
    dx, mm = GEAR_TIERS[tier]
    wl = synth.gear_workload(dx=dx, seed=3, samples_per_period=12, rings=4, move_mask=mm)
    print(f"[parity] gear tier {tier} dx={dx} n={wl.n} moving={wl.n_moving()}", flush=True)
    r = _relaxer(wl)
    r.build_cells()
    r.relax_step(count_pairs=True)
    acc = r.by_id(r.accel)
    mov = oforce.moving_mask(wl.tag, wl.move_mask)
    a64, S, cnt = oforce.accel(wl, receivers=np.nonzero(mov)[0])
    err = np.linalg.norm(acc[mov, :3].astype(np.float64) - a64, axis=1)
    assert np.all(err <= 1e-5 * S), float(np.max(err / np.maximum(S, 1e-300)))
    assert np.array_equal(acc[mov, 3].astype(np.int64), cnt)
    r2 = _relaxer(wl)
    r2.step()
    ref = ostep.relax_step(wl)
    _compare_step(wl, r2, ref)
    assert r2.read_status() == 0


def test_steps_keep_invariants_and_match_oracle_each_step():
    """Five iterations on the cube: every step from the GPU's own state is
    checked against the oracle applied to that same state, and the invariants
    hold (surface particles on their facet plane, features on their edge,
    volume particles inside)."""
    wl = synth.cube_workload(n=12, seed=9)
    r = _relaxer(wl)
    dx = wl.geoms[0].dx
    for it in range(5):
        pos, owner, fs, fu = r.host_state()
        ref = ostep.relax_step(wl, pos32=pos, owner=owner, feat_seg=fs, feat_u=fu)
        r.step()
        p2, o2 = _compare_step(wl, r, ref)
        x = p2.astype(np.float64)
        s = wl.tag == synth.SURFACE
        A, B, C, n = ogeo.facet_frames(wl.geoms[0].mesh.vert, wl.geoms[0].mesh.tri)
        d = np.einsum("ij,ij->i", x[s] - A[o2[s]], n[o2[s]])
        assert np.abs(d).max() <= 1e-6 * dx
        v = wl.tag == synth.VOLUME
        sd = ogeo.signed_distance_many(x[v], wl.geoms[0].mesh.vert, wl.geoms[0].mesh.tri)
        assert (sd < 0).all()


def test_determinism_bitwise():
    wl = synth.sphere_workload(level=3, dx=0.08, seed=2)
    outs = []
    for _ in range(2):
        r = _relaxer(wl)
        for _ in range(3):
            r.step()
        outs.append(r.host_state())
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_hvp_matches_oracle_jacobian():
    wl = synth.cube_workload(n=10, seed=12)
    r = _relaxer(wl)
    r.build_cells()
    rng = np.random.Generator(np.random.PCG64(13))
    v = rng.normal(size=(wl.n, 3))
    ids = r.id.cpu().numpy()
    v4 = np.zeros((wl.n, 4), np.float32)
    v4[:, :3] = v[ids]
    vt = torch.from_numpy(v4).cuda()
    for transpose in (False, True):
        out = r.by_id(r.hvp(vt, transpose=transpose))[:, :3].astype(np.float64)
        ref = ohvp.vjp(wl, v.astype(np.float32).astype(np.float64)) if transpose else \
            ohvp.jvp(wl, v.astype(np.float32).astype(np.float64))
        err = np.linalg.norm(out - ref, axis=1)
        scale = np.linalg.norm(ref, axis=1).max()
        assert err.max() <= 1e-4 * scale, (transpose, float(err.max() / scale))


def test_nonfinite_input_is_flagged_and_held():
    """A NaN position is never anyone's neighbour, is reported through the
    status word when it is moved, and leaves the other particles' forces equal
    to the oracle's."""
    wl = synth.cube_workload(n=8, seed=3)
    wl.pos[5] = np.nan
    r = _relaxer(wl)
    r.build_cells()
    r.relax_step()
    acc = r.by_id(r.accel)
    assert np.isfinite(acc).all()
    a64, S, _ = oforce.accel(wl)
    mov = oforce.moving_mask(wl.tag, wl.move_mask)
    mov[5] = False
    err = np.linalg.norm(acc[:, :3].astype(np.float64) - a64, axis=1)
    assert np.all(err[mov] <= 1e-5 * S[mov])
    r.project()
    assert r.read_status() & 2          # FPPG_S_NONFINITE_POS
    pos, _, _, _ = r.host_state()
    assert np.isnan(pos[5]).all() and np.isfinite(np.delete(pos, 5, 0)).all()


# --------------------------------------------------------------------------- degenerate inputs

def test_empty_workload_steps_cleanly():
    from synth import meshes as M
    wl = synth.workload.custom_workload(M.cube(), 0.05, np.zeros((0, 3)), np.zeros(0, np.int32))
    r = _relaxer(wl)
    for _ in range(2):
        r.step()
    assert r.read_status() == 0
    assert not r.counters.cpu().numpy().any()
    assert r.cell_start.cpu().numpy().max() == 0


def test_nothing_moves_when_the_move_mask_is_empty():
    wl = synth.cube_workload(n=8, seed=4, move_mask=0)
    r = _relaxer(wl)
    r.build_cells()
    before = r.pos.clone()
    r.relax_step()
    assert float(r.amax.cpu()[0]) == 0.0
    r.project()
    assert torch.equal(before, r.pos)
    assert r.read_status() == 0


def test_isolated_and_coincident_particles():
    """A lone particle feels nothing and does not move; two particles at the
    same point exert no force on each other (r = 0) but both feel a third."""
    from synth import meshes as M
    dx = 0.05
    p = np.array([[0.2, 0.2, 0.2], [0.6, 0.6, 0.6], [0.6, 0.6, 0.6], [0.62, 0.6, 0.6]])
    wl = synth.workload.custom_workload(M.cube(), dx, p, np.full(4, synth.VOLUME))
    r = _relaxer(wl)
    r.build_cells()
    r.relax_step(count_pairs=True)
    acc = r.by_id(r.accel)
    a64, S, cnt = oforce.accel(wl)
    assert np.array_equal(acc[:, 3].astype(np.int64), cnt) and cnt.tolist() == [0, 2, 2, 2]
    assert not acc[0, :3].any()
    err = np.linalg.norm(acc[:, :3].astype(np.float64) - a64, axis=1)
    assert np.all(err <= 1e-5 * np.maximum(S, 1e-30))
    v = np.zeros((4, 4), np.float32)
    v[:, :3] = np.random.Generator(np.random.PCG64(3)).normal(size=(4, 3))
    ids = r.id.cpu().numpy()
    vt = torch.from_numpy(v[ids]).cuda()
    for transpose in (False, True):
        out = r.by_id(r.hvp(vt, transpose=transpose))[:, :3].astype(np.float64)
        vd = v[:, :3].astype(np.float64)
        ref = ohvp.vjp(wl, vd) if transpose else ohvp.jvp(wl, vd)
        assert np.all(np.isfinite(out))
        assert np.abs(out - ref).max() <= 1e-4 * np.abs(ref).max()
    r.project()
    pos, _, _, _ = r.host_state()
    assert np.array_equal(pos[0], wl.pos[0])          # lone particle: a = 0
    assert r.read_status() == 0


def test_volume_moves_that_end_at_or_across_a_facet_plane_revert():
    """Prescribed displacements of volume particles a few ulps inside the
    cube's faces: a move is reverted exactly when its end point lies on or
    beyond the face (the binary32 plane prefilter defers every close call to
    the FP64 test)."""
    from synth import meshes as M
    one = np.float32(1.0)
    pts, moves = [], []
    for axis in range(3):
        for a in range(1, 7):
            for b in range(0, 9):
                p = np.full(3, np.float32(0.3) + np.float32(0.005 * (a + 7 * b)), np.float32)
                p[axis] = one
                for _ in range(a):
                    p[axis] = np.nextafter(p[axis], np.float32(0))
                y = p[axis]
                for _ in range(b):
                    y = np.nextafter(y, np.float32(2))
                d = np.zeros(3, np.float32)
                d[axis] = np.float32(y - p[axis])          # exact: both near 1
                pts.append(p)
                moves.append(d)
    p = np.array(pts, np.float32)
    dvec = np.array(moves, np.float32)
    wl = synth.workload.custom_workload(M.cube(), 0.05, p, np.full(len(p), synth.VOLUME))
    r = _relaxer(wl)
    r.build_cells()
    ids = r.id.cpu().numpy()
    disp = np.zeros((wl.n, 4), np.float32)
    disp[:, :3] = dvec[ids]
    r.disp.copy_(torch.from_numpy(disp))
    r.project()
    pos, _, _, _ = r.host_state()
    y = (p + dvec).astype(np.float32)
    outside = np.any(y >= one, axis=1)
    assert outside.any() and (~outside).any()
    assert np.array_equal(pos[outside], p[outside])
    assert np.array_equal(pos[~outside], y[~outside])
    assert int(r.counters.cpu()[2]) == int(outside.sum())


# --------------------------------------------------------------------------- error paths

def test_host_side_errors_with_a_live_context():
    """Argument errors are returned (and described) without launching anything."""
    import ctypes
    from paper_2501_03056_amd import _lib
    from paper_2501_03056_amd._lib import ptr
    from paper_2501_03056_amd.relax import geom_descs
    wl = synth.cube_workload(n=4, seed=2)
    r = _relaxer(wl)
    L, c, g = r.ctx.lib, r.ctx.handle, r.geom.handle
    st = r.stream
    # workspace too small
    assert L.fppg_build_cells(c, g, r.n, ptr(r.pos), ptr(r.id), ptr(r.owner), ptr(r.pos_b), ptr(r.id_b),
                              ptr(r.owner_b), ptr(r.cell_start), r.ws_ptr, 16, st) == _lib.E_WORKSPACE
    assert b"workspace" in L.fppg_last_error(c)
    # particle count differs from the geometry's
    assert L.fppg_relax_step(c, g, r.n + 1, ptr(r.pos), ptr(r.owner), ptr(r.cell_start), ptr(r.feat_seg),
                             r.n_feat, r.move_mask, 0, None, ptr(r.amax), ptr(r.disp), None, 0, r.ws_ptr,
                             r.ws_bytes, st) == _lib.E_ARG
    # a receiver list longer than the particle arrays
    assert L.fppg_relax_step(c, g, r.n, ptr(r.pos), ptr(r.owner), ptr(r.cell_start), ptr(r.feat_seg),
                             r.n_feat, r.move_mask, 0, None, ptr(r.amax), ptr(r.disp), ptr(r.mlist), r.n + 1,
                             r.ws_ptr, r.ws_bytes, st) == _lib.E_ARG
    # misaligned position array
    mis = ctypes.c_void_p(r.pos.data_ptr() + 4)
    assert L.fppg_project(c, g, r.n, mis, ptr(r.owner), ptr(r.disp), ptr(r.feat_seg), ptr(r.feat_u), r.n_feat,
                          r.move_mask, ptr(r.counters), None, 0, r.ws_ptr, r.ws_bytes, st) == _lib.E_ARG
    # aliasing input and output
    assert L.fppg_relax_hvp(c, g, r.n, ptr(r.pos), ptr(r.cell_start), r.move_mask, 0, ptr(r.disp), ptr(r.disp),
                            st) == _lib.E_ARG
    # an odd iteration count cannot be replayed back to back
    h = ctypes.c_void_p()
    side = torch.cuda.Stream()
    assert L.fppg_graph_create(c, g, r.n, ptr(r.pos), ptr(r.id), ptr(r.owner), ptr(r.pos_b), ptr(r.id_b),
                               ptr(r.owner_b), ptr(r.cell_start), ptr(r.feat_seg), ptr(r.feat_u), r.n_feat,
                               r.move_mask, ptr(r.amax), ptr(r.disp), ptr(r.counters), r.ws_ptr, r.ws_bytes, 3,
                               ctypes.c_void_p(side.cuda_stream), ctypes.byref(h)) == _lib.E_ARG
    # unsupported stencil half-width
    bad = synth.cube_workload(n=4, seed=2)
    bad.geoms[0].k = 3
    arr, keep = geom_descs(bad.geoms)
    assert L.fppg_geom_create(c, arr, 1, ctypes.byref(h)) == _lib.E_UNSUPPORTED
    # nothing above reached the device
    r.step()
    assert r.read_status() == 0


@pytest.mark.parametrize("tier", ["feature", "surface"])
def test_receiver_list_gives_the_same_iterations(tier):
    """Relaxing one class with the moving-particle list (only its lanes
    launched) gives bit for bit the state of the full launch."""
    mm = {"feature": 1 << synth.FEATURE, "surface": 1 << synth.SURFACE}[tier]
    wl = synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4, move_mask=mm)
    ra, rb = _relaxer(wl), _relaxer(wl)
    rb.use_list = True
    for _ in range(3):
        ra.step()
        rb.step()
    assert int(rb.mcount.cpu()[0]) == rb.n_moving() == wl.n_moving()
    ids = rb.mlist[: rb.n_moving()].cpu().numpy()
    assert np.all(np.diff(ids) > 0)
    sa, sb = ra.host_state(), rb.host_state()
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert torch.equal(ra.counters, rb.counters)
    assert ra.read_status() == 0 and rb.read_status() == 0


@pytest.mark.parametrize("n_clump,n_nan", [(65, 0), (4096, 0), (4097, 70), (20000, 0), (0, 9000), (9000, 5000)])
def test_cells_bit_exact_with_crowded_cells(n_clump, n_nan):
    """Cells of more than 64 particles (a clump inside one particle cell, the
    quarantine cell of the non-finite particles) are ordered by id like the
    others; the sizes cross the LDS chunk (4096) and need merge passes."""
    from synth import meshes as M
    base = synth.cube_workload(n=8, seed=1)
    rng = np.random.Generator(np.random.PCG64(n_clump + 7 * n_nan))
    centre = np.array([0.5, 0.5, 0.5]) + 0.01 * base.geoms[0].dx
    clump = centre + rng.uniform(-1e-4, 1e-4, size=(n_clump, 3)) * base.geoms[0].dx
    nan = np.full((n_nan, 3), np.nan)
    pos = np.concatenate([base.pos.astype(np.float64), clump, nan])
    tag = np.concatenate([base.tag, np.full(n_clump + n_nan, 3, np.int32)])
    perm = rng.permutation(len(pos))   # ids in no spatial order
    wl = synth.workload.custom_workload(M.cube(), base.geoms[0].dx, pos[perm], tag[perm])
    r = _relaxer(wl)
    r.build_cells()
    torch.cuda.synchronize()
    keys = ocells.cell_keys(wl)
    order = ocells.sort_order(keys, wl.ids)
    cs = ocells.cell_start(keys[order], ocells.total_cells(wl))
    occ = np.diff(cs)
    assert occ.max() > 64   # the clump's cell holds two lattice particles besides it
    assert np.array_equal(r.id.cpu().numpy(), order)
    assert np.array_equal(r.cell_start.cpu().numpy(), cs)
    got = r.pos.cpu().numpy()[:, :3]
    want = wl.pos[order]
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.array_equal(np.nan_to_num(got), np.nan_to_num(want))
    before = r.pos.clone()
    r.build_cells()
    assert torch.equal(before.nan_to_num(), r.pos.nan_to_num())
