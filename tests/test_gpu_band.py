"""Three-layer volume relaxation on the GPU (section 3.3.4): fppg_volume_layers
against the oracle's layer split, one relaxation step of the layered workload
against the FP64 oracle, and the volume tier of the layered workload with and
without the receiver list."""
import copy

import numpy as np
import pytest

import synth
from oracle import band as oband
from oracle import step as ostep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _relaxer(wl):
    from paper_2501_03056_amd import Relaxer
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Relaxer(wl, device=0)


def _device_tags(r):
    w = r.by_id(r.pos)[:, 3].copy()
    return w.view(np.int32) & 7


def _distance(wl):
    d = np.full(wl.n, np.inf)
    for g, geo in enumerate(wl.geoms):
        sel = np.flatnonzero(wl.gid == g)
        d[sel] = oband.surface_distance(wl.pos[sel].astype(np.float32).astype(np.float64),
                                        geo.mesh.vert, geo.mesh.tri)
    return d


CASES = {
    "cube_n12": (lambda: synth.cube_workload(n=12, seed=3), 2.5 / 12),
    "sphere_l3": (lambda: synth.sphere_workload(level=3, dx=0.08, seed=2), 0.2),
    "batch3": (lambda: synth.workload.solid_batch_workload(n_geom=3, n_min=3000, n_max=8000, seed=21), None),
    "gear_coarse": (lambda: synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4), 0.1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_layer_tags_match_oracle(case):
    make, W = CASES[case]
    wl = make()
    if W is None:
        W = 3.0 * float(wl.geoms[0].dx)
    r = _relaxer(wl)
    k = r.volume_layers(W)
    want = oband.layer_tags(wl, W)
    got = _device_tags(r)
    d = _distance(wl)
    clear = np.abs(d - W) > 1e-9 * W   # a distance this close to W may round either way
    assert np.array_equal(got[clear], want[clear])
    assert k == int(np.sum((got == synth.FIXED) & (wl.tag == synth.VOLUME)))
    assert k == int(np.sum(want == synth.FIXED) - np.sum(wl.tag == synth.FIXED)) or not clear.all()
    assert 0 < k < int(np.sum(wl.tag == synth.VOLUME))
    assert r.n_moving() == int(np.sum((wl.move_mask >> got) & 1))
    assert r.read_status() == 0


def test_width_zero_fixes_every_volume_particle():
    wl = synth.cube_workload(n=8, seed=4)
    r = _relaxer(wl)
    assert r.volume_layers(0.0) == int(np.sum(wl.tag == synth.VOLUME))
    assert not np.any(_device_tags(r) == synth.VOLUME)


def test_layered_step_matches_oracle():
    wl = synth.sphere_workload(level=3, dx=0.08, seed=2)
    W = 0.2
    r = _relaxer(wl)
    r.volume_layers(W)
    wl2 = copy.copy(wl)
    wl2.tag = _device_tags(r)   # the split itself is checked above
    r.step()
    ref = ostep.relax_step(wl2)
    pos, _, _, _ = r.host_state()
    ok = ~ref.margin
    x = ref.pos32.astype(np.float64)
    tol = 1e-5 * np.maximum(np.abs(x).max(1), wl.geoms[0].dx)
    err = np.abs(pos.astype(np.float64) - x).max(1)
    assert not (ok & (err > tol)).any(), float(err[ok].max())
    core = wl2.tag == synth.FIXED
    assert np.array_equal(pos[core], wl.pos[core].astype(np.float32))   # the core does not move
    assert r.read_status() == 0


def test_layered_volume_tier_with_receiver_list_is_bitwise_equal():
    wl = synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4, move_mask=1 << synth.VOLUME)
    ra, rb = _relaxer(wl), _relaxer(wl)
    W = 0.1
    assert ra.volume_layers(W) == rb.volume_layers(W)
    rb.use_list = True
    for _ in range(3):
        ra.step()
        rb.step()
    assert int(rb.mcount.cpu()[0]) == rb.n_moving() < wl.n_moving()
    for x, y in zip(ra.host_state(), rb.host_state()):
        assert np.array_equal(x, y)
    assert torch.equal(ra.counters, rb.counters)
