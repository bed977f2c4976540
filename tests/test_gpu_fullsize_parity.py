"""GPU parity at the benchmark sizes, element by element against the oracle's
full-size mode (oracle/local.py, pinned to the brute-force oracle by
tests/test_oracle_local.py):

  * the sphere (icosphere level 5, dx = 0.01, 4.25 M particles): one step,
    every particle
  * the gear on its full mesh (207,360 facets, side walls of aspect ~70 and
    ~340, dx = 0.004, 12.4 M particles): one step of each tier (feature lines,
    surfaces, volume), every moving particle, with the oracle's own amax
  * the three largest Boolean assemblies of the 64-assembly batch and its two
    largest differences (1.7 M particles, every class moving), one step in the
    benchmark's tuned launch: forces and amax of every particle, every
    surface and feature particle and a sample of the volume particles
  * particles forced to revert (feature particles off open line ends, surface
    particles off their facet, volume particles pushed out through the skin)
    on the cube, the tetrahedron, the sphere and the gear
  * the cube of dx = 1/24: 100 iterations with the invariants after every
    step and the oracle's step from the GPU's state every 10th

Bars: positions within 1e-5 max(|x|, dx) of the oracle's binary32 result,
owners and feature segments equal, revert counts per class equal, for every
particle whose decision is not within rounding of flipping (the oracle flags
those as margin; at most 0.1 % of the movers, and they still satisfy the
invariants).
"""
import copy

import numpy as np
import pytest

import synth
from facet_bound import assert_on_facets
from oracle import force as oforce
from oracle import local as olocal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _relaxer(wl):
    from paper_2501_03056_amd import Relaxer
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Relaxer(wl, device=0)


def _compare(wl, r, ref, label, max_margin=1e-3, sample=None):
    """Positions, owners, feature tables and revert counts of the GPU's step
    against the oracle's; returns (GPU positions, owners, margin count).
    max_margin: the largest fraction of the movers that may be margin cases.
    sample: the particles the oracle projected (relax_step's sample); revert
    counts are compared for the classes it covers entirely."""
    pos, owner, fs, fu = r.host_state()
    sample = np.ones(wl.n, bool) if sample is None else np.asarray(sample, bool)
    mov = oforce.moving_mask(wl.tag, wl.move_mask) & sample
    ok = ~ref.margin & sample
    n_margin = int(np.sum(ref.margin & mov))
    assert n_margin <= max(1, max_margin * mov.sum()), (label, n_margin, int(mov.sum()))
    x = ref.pos32.astype(np.float64)
    dx = np.array([g.dx for g in wl.geoms])[wl.gid]   # each particle's geometry spacing
    tol = 1e-5 * np.maximum(np.abs(x).max(1), dx)
    err = np.abs(pos.astype(np.float64) - x).max(1)
    bad = ok & (err > tol)
    assert not bad.any(), (label, int(bad.sum()), np.nonzero(bad)[0][:10], float(err[ok].max()))
    s = ok & (wl.tag == synth.SURFACE)
    assert np.array_equal(owner[s], ref.owner[s]), label
    f = np.nonzero(ok & (wl.tag == synth.FEATURE))[0]
    if len(f):
        slots = wl.owner[f]
        assert np.array_equal(fs[slots], ref.feat_seg[slots]), label
        assert np.all(np.abs(fu[slots] - ref.feat_u[slots]) <= 1e-5 * dx[f]), label
    c = r.counters.cpu().numpy()
    all_mov = oforce.moving_mask(wl.tag, wl.move_mask)
    for k, tg in ((0, synth.SURFACE), (1, synth.FEATURE), (2, synth.VOLUME)):
        if np.any(all_mov & (wl.tag == tg) & ~sample):
            continue   # class sampled: its total is not the oracle's
        m = mov & (wl.tag == tg)
        want = int(np.sum(ref.reverted & m))
        slack = int(np.sum(ref.margin & m))
        assert abs(int(c[k]) - want) <= slack, (label, tg, int(c[k]), want, slack)
    # the margin particles still satisfy the invariants
    for g, geo in enumerate(wl.geoms):
        sm = ref.margin & (wl.tag == synth.SURFACE) & (wl.gid == g)
        if sm.any():
            assert_on_facets(pos[sm], geo.mesh, owner[sm] - geo.tri_begin, geo.dx)
    print(f"[fullsize] {label}: {int(mov.sum())} movers checked, {int(np.sum(ref.reverted & mov))} reverted, "
          f"{n_margin} margin, max position error {float(err[ok & mov].max()) if np.any(ok & mov) else 0.0:.3g}",
          flush=True)
    return pos, owner, n_margin


def test_full_sphere_one_step_every_particle():
    wl = synth.sphere_workload(level=5, dx=0.01, seed=2)
    print(f"[fullsize] sphere l5 dx=0.01: {wl.n} particles", flush=True)
    r = _relaxer(wl)
    r.step()
    torch.cuda.synchronize()
    ref = olocal.relax_step(wl)
    amax = r.amax.cpu().numpy()
    assert np.allclose(amax, ref.amax, rtol=1e-5)
    pos, owner, _ = _compare(wl, r, ref, "sphere")
    s = wl.tag == synth.SURFACE
    assert_on_facets(pos[s], wl.geoms[0].mesh, owner[s], wl.geoms[0].dx)
    assert r.read_status() == 0


@pytest.fixture(scope="module")
def gear_full():
    return synth.gear_workload(dx=0.004, seed=3)


@pytest.mark.parametrize("tier", ["feature", "surface", "volume"])
def test_full_gear_tier_one_step_every_mover(gear_full, tier):
    """One step of a tier of the gear on its full mesh: the tier partition, the
    receiver list of a sparse tier and the full launch of the volume tier, each
    against the oracle's step over all particles (its own forces and amax)."""
    mm = {"feature": 1 << synth.FEATURE, "surface": 1 << synth.SURFACE, "volume": 1 << synth.VOLUME}[tier]
    wl = copy.copy(gear_full)
    wl.move_mask = mm
    mesh = wl.geoms[0].mesh
    print(f"[fullsize] gear dx=0.004 tier {tier}: {wl.n} particles, {wl.n_moving()} moving, "
          f"{len(mesh.tri)} facets", flush=True)
    r = _relaxer(wl)
    r.tier(mm)
    r.use_list = wl.n_moving() < r.na // 2
    r.step()
    torch.cuda.synchronize()
    ref = olocal.relax_step(wl)
    assert np.allclose(r.amax.cpu().numpy(), ref.amax, rtol=1e-5)
    pos, owner, _ = _compare(wl, r, ref, f"gear {tier}")
    if tier == "surface":
        s = np.nonzero(wl.tag == synth.SURFACE)[0]
        assert_on_facets(pos[s], mesh, owner[s], wl.geoms[0].dx)
        # the near-degenerate side walls (vertical facets of aspect ~70 and ~340) are covered
        A, B, C = (mesh.vert[mesh.tri[owner[s], q]] for q in range(3))
        nz = np.cross(B - A, C - A)[:, 2]
        wall = np.abs(nz) < 1e-12
        rad = np.hypot(pos[s, 0], pos[s, 1])
        assert wall.sum() > 1000 and np.sum(wall & (rad < 0.25)) > 100, (int(wall.sum()), int(np.sum(wall & (rad < 0.25))))
    assert r.read_status() == 0


def test_full_gear_volume_tier_is_the_same_in_every_xcd_mapping(gear_full):
    """The launch the benchmark times on the gear (256 threads, runs of 16
    chunks dealt to the XCDs in turn: of 48,264 chunks all but the last 8,
    the rest of a round of 8 runs, are in runs) and the other two XCD
    mappings give the same two
    volume-tier iterations and the same Jacobian product, bit for bit."""
    wl = copy.copy(gear_full)
    wl.move_mask = 1 << synth.VOLUME
    v = np.random.default_rng(11).standard_normal((wl.n, 4)).astype(np.float32)
    ref = None
    for remap in (1, 2, 0):
        print(f"[fullsize] gear volume tier, XCD mapping {remap}", flush=True)
        r = _relaxer(wl)
        r.tier(wl.move_mask)
        r.ctx.set_launch(256, remap, False)
        for _ in range(2):
            r.step()
        r.build_cells()
        jv = r.hvp(torch.from_numpy(v[:r.na]).to(r.pos.device)).cpu().numpy()
        got = [*r.host_state(), r.amax.cpu().numpy(), jv]
        assert r.read_status() == 0
        del r
        if ref is None:
            ref = got
            continue
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), remap


def test_largest_batch_assemblies_one_step_every_mover():
    """The three largest Boolean assemblies of the 64-assembly benchmark batch
    (seed 4000, all unions) and its two largest differences (each built exactly
    as in the batch, every class moving; 1.7 M particles), one
    step in the benchmark's tuned launch (stencil k = 2, 512-thread force
    blocks, XCD-contiguous chunks, eager) against the oracle's step (its own
    forces and amax per geometry over every particle; every surface and
    feature particle and a seeded sample of the volume particles projected)."""
    targets = synth.workload.batch_targets(64, 5e3, 5e5, 4000)
    members = [5, 22, 53, 55, 61]
    assert sorted(np.argsort(targets)[-3:].tolist()) == members[:3]
    print(f"[fullsize] batch members {members}: targets {[round(targets[b]) for b in members]}", flush=True)
    wl = synth.workload.batch_workload(n_geom=64, seed=4000, members=members)
    ops = [a["op"] for a in wl.meta["assemblies"]]
    print(f"[fullsize] built {wl.n} particles, ops {ops}", flush=True)
    assert ops == ["union"] * 3 + ["difference"] * 2 and wl.n > 1_500_000
    r = _relaxer(wl)
    r.ctx.set_launch(512, True, False)
    r.step()
    torch.cuda.synchronize()
    print("[fullsize] batch members: GPU step done", flush=True)
    # forces and amax of every particle; every surface, feature and singular
    # particle projected, and 40,000 volume particles (the CSG volume rule is
    # a brute-force distance over the parts' facets)
    rng = np.random.default_rng(11)
    vol = np.nonzero(wl.tag == synth.VOLUME)[0]
    sample = wl.tag != synth.VOLUME
    sample[rng.choice(vol, 40_000, replace=False)] = True
    ref = olocal.relax_step(wl, sample=sample)
    print("[fullsize] batch members: oracle step done", flush=True)
    assert np.allclose(r.amax.cpu().numpy(), ref.amax, rtol=1e-5)
    pos, owner, _ = _compare(wl, r, ref, "batch members", sample=sample)
    for g, geo in enumerate(wl.geoms):
        s = np.nonzero((wl.tag == synth.SURFACE) & (wl.gid == g))[0]
        assert_on_facets(pos[s], geo.mesh, owner[s] - geo.tri_begin, geo.dx)
    assert r.read_status() == 0


FORCED = {
    "cube": lambda: synth.workload.forced_reverts(synth.cube_workload(n=10, seed=3), seed=1),
    "tetra": lambda: synth.workload.forced_reverts(synth.tetra_workload(dx=0.06, seed=5), seed=2),
    "sphere_l3": lambda: synth.workload.forced_reverts(synth.sphere_workload(level=3, dx=0.08, seed=2), seed=3),
    "gear_all_classes": lambda: synth.workload.forced_reverts(
        synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4), seed=5),
    "gear_full_mesh_surface": lambda: synth.workload.forced_reverts(
        synth.gear_workload(dx=0.01, seed=3, move_mask=(1 << synth.SURFACE) | (1 << synth.FEATURE)), seed=6),
}


@pytest.mark.parametrize("case", list(FORCED))
def test_forced_reverts_match_oracle(case):
    wl = FORCED[case]()
    print(f"[fullsize] forced reverts {case}: {wl.n} particles", flush=True)
    r = _relaxer(wl)
    r.step()
    torch.cuda.synchronize()
    ref = olocal.relax_step(wl)
    mov = oforce.moving_mask(wl.tag, wl.move_mask)
    for tg in (synth.FEATURE, synth.SURFACE, synth.VOLUME):
        if np.any(mov & (wl.tag == tg)):
            assert ref.reverted[mov & (wl.tag == tg)].sum() >= 1, (case, tg)
    _compare(wl, r, ref, f"forced {case}")
    assert r.read_status() == 0


def test_cube_hundred_iterations_invariants_and_oracle_every_tenth():
    """The cube of dx = 1/24 (13,824 volume + 3,456 surface + 276 feature + 8
    singular particles, all classes moving): 100 iterations. After every step:
    surface particles on their facet (binary32 bound), feature particles on
    their edge, every volume particle strictly inside the cube, nothing lost.
    Before every 10th step: the oracle's step from the GPU's state."""
    wl = synth.cube_workload(n=24, seed=1)
    r = _relaxer(wl)
    dx = wl.geoms[0].dx
    mesh = wl.geoms[0].mesh
    s = wl.tag == synth.SURFACE
    f = np.nonzero(wl.tag == synth.FEATURE)[0]
    v = wl.tag == synth.VOLUME
    seg_p = mesh.lines.seg_p
    checked = 0
    for it in range(100):
        if it % 10 == 0:
            pos, owner, fs, fu = r.host_state()
            ref = olocal.relax_step(wl, pos32=pos, owner=owner, feat_seg=fs, feat_u=fu)
            r.counters.zero_()   # revert counts of this step only
            r.step()
            # as the surface particles relax they gather along the cube's edges and
            # cross the diagonals splitting each face into two coplanar facets: foot
            # points within 1e-7 (barycentric) of a facet edge are margin cases
            # (0.03 % after 10 iterations, 0.12 % after 20, 0.23 % after 30 on the
            # oracle's own trajectory), so the long run allows 0.5 %
            _compare(wl, r, ref, f"cube iteration {it}", max_margin=5e-3)
            checked += 1
        else:
            r.step()
        pos, owner, fs, fu = r.host_state()
        assert np.all(np.isfinite(pos))
        assert_on_facets(pos[s], mesh, owner[s], dx)
        # feature particles on the segment their slot records (the cube's edges are axis-aligned)
        sg = fs[wl.owner[f]]
        a, b = seg_p[sg, 0], seg_p[sg, 1]
        d = np.linalg.norm(np.cross(pos[f].astype(np.float64) - a, b - a), axis=1) / np.linalg.norm(b - a, axis=1)
        assert d.max() <= 1e-7, (it, float(d.max()))
        assert np.all((pos[v] > 0) & (pos[v] < 1)), it
    assert checked == 10
    assert r.read_status() == 0
