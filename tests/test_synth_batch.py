"""The batch builder: a member built alone is the same geometry and the same
particles as in the whole batch, and the targets are the batch's."""
import numpy as np

from synth import workload as W


def test_members_are_built_as_in_the_whole_batch():
    kw = dict(n_geom=3, n_min=1e3, n_max=2e3, seed=77, mc_samples=20_000)
    full = W.batch_workload(**kw)
    one = W.batch_workload(members=[2], **kw)
    g = full.geoms[2]
    sl = slice(g.part_begin, g.part_end)
    assert one.n == g.part_end - g.part_begin
    assert np.array_equal(one.pos, full.pos[sl])
    assert np.array_equal(one.tag, full.tag[sl])
    assert np.array_equal(one.geoms[0].mesh.vert, g.mesh.vert)
    assert np.array_equal(one.geoms[0].mesh.tri, g.mesh.tri)
    assert one.meta["assemblies"][0] == full.meta["assemblies"][2]
    assert W.batch_targets(3, 1e3, 2e3, 77) == full.meta["targets"]
