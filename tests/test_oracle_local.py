"""Pins of the oracle's full-size mode (oracle/local.py) against the
brute-force oracle: the candidate searches must not change a single decision.

  * forces over grid candidates = forces over all pairs (same source counts,
    sums equal up to summation order)
  * one whole step (forces, amax, time step, projection, feature walk, volume
    rule, margins) = the brute-force step on cubes, the icosphere, the
    tetrahedron and the gear tiers, including forced reverts
  * the vertical-ray winding number = the solid-angle winding number
  * the facet grid holds every facet within its pad of a point
"""
import numpy as np
import pytest

import synth
from synth import meshes as M
from oracle import force, geometry, local, step

CASES = {
    "cube_n12": lambda: synth.cube_workload(n=12, seed=31),
    "cube_n10_k1": lambda: synth.cube_workload(n=10, seed=7, k=1),
    "sphere_l3": lambda: synth.sphere_workload(level=3, dx=0.08, seed=2),
    "tetra": lambda: synth.tetra_workload(dx=0.06, seed=5),
    "gear_feature": lambda: synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4,
                                                move_mask=1 << synth.FEATURE),
    "gear_surface": lambda: synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4,
                                                move_mask=1 << synth.SURFACE),
    "gear_volume": lambda: synth.gear_workload(dx=0.06, seed=3, samples_per_period=12, rings=4,
                                               move_mask=1 << synth.VOLUME),
}


@pytest.mark.parametrize("case", ["cube_n12", "sphere_l3", "tetra", "gear_surface", "gear_volume"])
def test_candidate_forces_equal_brute_force(case):
    wl = CASES[case]()
    a0, S0, c0 = force.accel(wl)
    a1, S1, c1 = local.accel(wl, threads=3)
    assert np.array_equal(c0, c1)
    assert np.all(np.linalg.norm(a1 - a0, axis=1) <= 1e-13 * np.maximum(S0, 1e-300))
    assert np.allclose(S1, S0, rtol=1e-13, atol=0)


def _same_step(a, b):
    assert np.array_equal(a.reverted, b.reverted)
    assert np.array_equal(a.margin, b.margin)
    assert np.array_equal(a.owner, b.owner)
    assert np.array_equal(a.feat_seg, b.feat_seg)
    assert np.allclose(a.feat_u, b.feat_u, rtol=1e-12, atol=1e-15)
    assert np.allclose(a.amax, b.amax, rtol=1e-13)
    # FP64 positions agree to the rounding of the force sums' order
    assert np.allclose(a.x_new, b.x_new, rtol=0, atol=1e-12 * max(1.0, float(np.abs(a.x_new).max())))


@pytest.mark.parametrize("case", list(CASES))
def test_local_step_equals_brute_force_step(case):
    wl = CASES[case]()
    ref = step.relax_step(wl)
    got = local.relax_step(wl)
    _same_step(got, ref)


def test_sampled_step_equals_the_full_step_on_the_sample():
    """A sampled step (an assembly of the batch, every class moving) decides
    the sampled movers as the full step does and leaves the others in place."""
    wl = synth.workload.batch_workload(n_geom=2, n_min=1.5e3, n_max=3e3, seed=4212, mc_samples=50_000)
    full = local.relax_step(wl)
    sample = np.random.default_rng(0).random(wl.n) < 0.3
    got = local.relax_step(wl, sample=sample)
    mov = force.moving_mask(wl.tag, wl.move_mask)
    on = sample & mov
    assert on.sum() > 100 and (~sample & mov).sum() > 100
    assert np.array_equal(got.pos32[on], full.pos32[on])
    assert np.array_equal(got.reverted[on], full.reverted[on])
    assert np.array_equal(got.owner[on], full.owner[on])
    assert np.array_equal(got.pos32[~on], wl.pos[~on])
    assert not got.reverted[~on].any() and not got.margin[~on].any()
    assert np.array_equal(got.amax, full.amax)


FORCED = {
    "cube": lambda: synth.workload.forced_reverts(synth.cube_workload(n=10, seed=3), seed=1),
    "tetra": lambda: synth.workload.forced_reverts(synth.tetra_workload(dx=0.06, seed=5), seed=2),
    "sphere_l3": lambda: synth.workload.forced_reverts(synth.sphere_workload(level=3, dx=0.08, seed=2), seed=3),
    "gear_feature": lambda: synth.workload.forced_reverts(
        synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4, move_mask=1 << synth.FEATURE), seed=4),
    "gear_surface": lambda: synth.workload.forced_reverts(
        synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4, move_mask=1 << synth.SURFACE), seed=5),
}


@pytest.mark.parametrize("case", list(FORCED))
def test_local_step_with_forced_reverts(case):
    """Particles placed where the step must revert (feature particles at the
    start of open lines, surface particles lifted off their facet, volume
    particles at the skin pushed out by the volume): every class that moves
    reverts, and the full-size mode decides every particle as brute force does."""
    wl = FORCED[case]()
    ref = step.relax_step(wl)
    mov = force.moving_mask(wl.tag, wl.move_mask)
    for tg in (synth.FEATURE, synth.SURFACE, synth.VOLUME):
        if np.any(mov & (wl.tag == tg)):
            assert ref.reverted[wl.tag == tg].sum() >= 1, tg
    got = local.relax_step(wl)
    _same_step(got, ref)


@pytest.mark.parametrize("mesh_name", ["cube", "sphere", "gear", "tetra"])
def test_ray_winding_equals_solid_angle_winding(mesh_name):
    mesh = {"cube": M.cube, "sphere": lambda: M.icosphere(3), "tetra": M.tetrahedron,
            "gear": lambda: M.gear(samples_per_period=12, rings=4)}[mesh_name]()
    lo, hi = mesh.bbox()
    rng = np.random.Generator(np.random.PCG64(11))
    p = rng.uniform(lo - 0.1, hi + 0.1, size=(3000, 3))
    # include points on shared edges' vertical lines (the fallback path) and near the surface
    p[:50, :2] = mesh.vert[rng.integers(len(mesh.vert), size=50), :2]
    wn = geometry.winding_number(p, mesh.vert, mesh.tri)
    d = geometry.unsigned_distance_many(p, mesh.vert, mesh.tri)
    far = d > 1e-9
    got = local.ray_winding(p, mesh.vert, mesh.tri)
    assert np.array_equal(got[far] > 0.5, wn[far] > 0.5)
    assert np.allclose(got[far], np.round(wn[far]), atol=1e-9)


def test_facet_grid_holds_every_facet_within_its_pad():
    mesh = M.gear(samples_per_period=12, rings=4)
    pad = 0.03
    grid = local.FacetGrid(mesh.vert, mesh.tri, pad)
    rng = np.random.Generator(np.random.PCG64(12))
    lo, hi = mesh.bbox()
    p = rng.uniform(lo - 0.05, hi + 0.05, size=(400, 3))
    # exact point-facet distances, one facet at a time over all points
    D = np.stack([geometry.unsigned_distance_many(p, mesh.vert, mesh.tri[t:t + 1]) for t in range(len(mesh.tri))], 1)
    seen = 0
    for pts, fac in grid.groups(p):
        fac = set(fac.tolist())
        for i in pts:
            near = set(np.nonzero(D[i] <= pad)[0].tolist())
            assert near <= fac
            seen += len(near)
    assert seen > 100
