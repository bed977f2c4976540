"""Tier partition on the GPU (fppg_tier_partition): the particles a tier
reaches (rank at most its highest moving class) are moved in front, the rest
is left out of the per-iteration calls, and the relaxation of the tier is bit
for bit that of the calls on all particles."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TIERS = {"feature": 1 << synth.FEATURE, "surface": 1 << synth.SURFACE}
RANK = np.array([0, 1, 2, 3, 3, 7, 7, 7])


def _relaxer(wl):
    from paper_2501_03056_amd import Relaxer
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Relaxer(wl, device=0)


def _gear(mm):
    return synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4, move_mask=mm)


@pytest.mark.parametrize("tier", list(TIERS))
def test_partition_is_stable_and_complete(tier):
    mm = TIERS[tier]
    r = _relaxer(_gear(mm))
    r.build_cells()
    torch.cuda.synchronize()
    id0 = r.id.cpu().numpy()
    pos0 = r.pos.cpu().numpy()
    rank0 = RANK[pos0[:, 3].view(np.int32) & 7]
    R = 1 if tier == "feature" else 2
    na = r.tier(mm)
    torch.cuda.synchronize()
    assert na == int(np.sum(rank0 <= R)) and 0 < na < r.n
    want = np.concatenate([id0[rank0 <= R], id0[rank0 > R]])
    assert np.array_equal(r.id.cpu().numpy(), want)
    assert np.array_equal(r.pos.cpu().numpy().view(np.int32),
                          np.concatenate([pos0[rank0 <= R], pos0[rank0 > R]]).view(np.int32))
    # the tail is in both buffers
    for a, b in ((r.pos, r.pos_b), (r.id, r.id_b), (r.owner, r.owner_b)):
        assert torch.equal(a[na:], b[na:])
    # the volume tier reaches every particle and keeps the order
    assert r.tier(1 << synth.VOLUME) == r.n
    assert np.array_equal(r.id.cpu().numpy(), want)


@pytest.mark.parametrize("use_list", [False, True])
@pytest.mark.parametrize("tier", list(TIERS))
def test_compacted_tier_matches_the_full_tier(tier, use_list):
    mm = TIERS[tier]
    wl = _gear(mm)
    ra, rb = _relaxer(wl), _relaxer(wl)
    ra.use_list = rb.use_list = use_list
    ra.step()
    rb.step()
    rb.tier(mm)
    assert rb.na < rb.n
    for _ in range(3):
        ra.step()
        rb.step()
    sa, sb = ra.host_state(), rb.host_state()
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert torch.equal(ra.counters, rb.counters)
    assert torch.equal(ra.amax, rb.amax)
    assert ra.read_status() == 0 and rb.read_status() == 0


def test_tiers_in_sequence_match_uncompacted_tiers():
    """feature -> surface -> volume, compacted against not: the same state."""
    wl = _gear(TIERS["feature"])
    ra, rb = _relaxer(wl), _relaxer(wl)
    for mm in (TIERS["feature"], TIERS["surface"], 1 << synth.VOLUME):
        ra.tier(mm, compact=False)
        rb.tier(mm)
        assert ra.na == ra.n
        for _ in range(2):
            ra.step()
            rb.step()
    assert rb.na == rb.n
    for x, y in zip(ra.host_state(), rb.host_state()):
        assert np.array_equal(x, y)
    assert ra.read_status() == 0 and rb.read_status() == 0


def test_batch_surface_tier_compacted():
    wl = synth.workload.batch_workload(n_geom=4, n_min=2e3, n_max=2e4, seed=11, move_mask=TIERS["surface"])
    ra, rb = _relaxer(wl), _relaxer(wl)
    rb.tier(TIERS["surface"])
    for _ in range(3):
        ra.step()
        rb.step()
    for x, y in zip(ra.host_state(), rb.host_state()):
        assert np.array_equal(x, y)
    assert torch.equal(ra.amax, rb.amax)


def test_calls_with_the_full_count_are_refused_while_compacted():
    from paper_2501_03056_amd import _lib
    r = _relaxer(_gear(TIERS["surface"]))
    r.tier(TIERS["surface"])
    na, r.na = r.na, r.n
    with pytest.raises(_lib.FppgError) as e:
        r.build_cells()
    assert e.value.status == _lib.E_ARG
    r.na = na
    r.step()
    assert r.read_status() == 0


@pytest.mark.parametrize("mm", [0, (1 << synth.FEATURE) | (1 << synth.SURFACE)])
def test_partition_of_no_mover_and_of_two_classes(mm):
    """No moving class: every particle stays active, in order. Feature and
    surface classes moving together: the tier reaches ranks 0..2."""
    r = _relaxer(_gear(TIERS["surface"]))
    r.build_cells()
    torch.cuda.synchronize()
    id0 = r.id.cpu().numpy()
    rank0 = RANK[r.pos.cpu().numpy()[:, 3].view(np.int32) & 7]
    na = r.tier(mm)
    if mm == 0:
        assert na == r.n
        assert np.array_equal(r.id.cpu().numpy(), id0)
    else:
        assert na == int(np.sum(rank0 <= 2))
        assert np.array_equal(r.id.cpu().numpy()[:na], id0[rank0 <= 2])
    r.step()
    assert r.read_status() == 0


def test_graph_replay_of_a_compacted_tier_with_a_launch_shape_equals_eager():
    """A HIP graph captured after the tier partition and a launch-shape change
    replays bit for bit the eager iterations of the same compacted tier."""
    mm = TIERS["surface"]
    wl = _gear(mm)
    eager, g = _relaxer(wl), _relaxer(wl)
    for r in (eager, g):
        r.step()
        r.tier(mm)
        r.ctx.set_launch(128, False)
    for _ in range(4):
        eager.step(keep_accel=False)
    g.capture(iters=2)
    g.replay(2)
    for a, b in zip(g.host_state(), eager.host_state()):
        assert np.array_equal(a, b)
    assert g.read_status() == 0
    g.release_graph()
