"""GPU parity at the benchmark's full size (icosphere level 5, dx = 0.01,
4,248,406 particles, stencil k = 2: the configuration bench.py times), on
what the oracle can compute at that size: the whole cell order (O(N) keys and
a sort), forces and neighbour counts of sampled receivers (brute force over
all N sources each), and properties of one step that hold at any size."""
import numpy as np
import pytest

import synth
from facet_bound import assert_on_facets
from oracle import cells as ocells
from oracle import force as oforce

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sphere():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return synth.sphere_workload(level=5, dx=0.01, seed=2)


def _relaxer(wl):
    from paper_2501_03056_amd import Relaxer
    return Relaxer(wl, device=0)


def test_full_size_cell_order_bit_exact(sphere):
    wl = sphere
    r = _relaxer(wl)
    r.build_cells()
    keys = ocells.cell_keys(wl)
    order = ocells.sort_order(keys, wl.ids)
    cs = ocells.cell_start(keys[order], ocells.total_cells(wl))
    assert np.array_equal(r.id.cpu().numpy(), order)
    assert np.array_equal(r.cell_start.cpu().numpy(), cs)


def test_full_size_sampled_forces_and_neighbour_counts(sphere):
    wl = sphere
    r = _relaxer(wl)
    r.build_cells()
    r.relax_step(count_pairs=True)
    acc = r.by_id(r.accel)
    rng = np.random.Generator(np.random.PCG64(7))
    surf = np.nonzero(wl.tag == synth.SURFACE)[0]
    sel = np.concatenate([rng.choice(wl.n, 64, replace=False), rng.choice(surf, 32, replace=False)])
    a64, S, cnt = oforce.accel(wl, receivers=sel)
    err = np.linalg.norm(acc[sel, :3].astype(np.float64) - a64, axis=1)
    assert np.all(err <= 1e-5 * S), float(np.max(err / S))
    assert np.array_equal(acc[sel, 3].astype(np.int64), cnt)
    amax = float(r.amax.cpu().numpy()[0])
    assert amax >= np.linalg.norm(a64, axis=1).max() * (1 - 1e-5)
    assert r.read_status() == 0


def test_full_size_one_step_properties(sphere):
    """One iteration: every move is at most h/16; accepted volume moves are
    dt^2 a with one dt^2 for all (checked against the oracle's a on sampled
    particles); surface particles stay on their owner facet."""
    wl = sphere
    r = _relaxer(wl)
    r.step()
    pos, owner, _, _ = r.host_state()
    h = float(wl.geoms[0].h)
    d = pos.astype(np.float64) - wl.pos.astype(np.float64)
    step = np.linalg.norm(d, axis=1)
    vol = wl.tag == synth.VOLUME
    assert step[vol].max() <= h / 16 * (1 + 1e-4)
    rng = np.random.Generator(np.random.PCG64(8))
    cand = np.nonzero(vol & (step > 0))[0]
    sel = rng.choice(cand, 48, replace=False)
    a64, _, _ = oforce.accel(wl, receivers=sel)
    # one dt^2 for all: d = dt^2 a up to the binary32 rounding of the new position
    tau = np.median(np.linalg.norm(d[sel], axis=1) / np.linalg.norm(a64, axis=1))
    ulp = np.spacing(np.abs(pos[sel]).astype(np.float32)).astype(np.float64)
    dev = np.abs(d[sel] - tau * a64)
    assert np.all(dev <= 1.01 * ulp + 1e-5 * np.abs(tau * a64).max(1, keepdims=True)), float(np.max(dev / ulp))
    mesh = wl.geoms[0].mesh
    s = np.nonzero(wl.tag == synth.SURFACE)[0]
    assert_on_facets(pos[s], mesh, owner[s], wl.geoms[0].dx)
    assert r.read_status() == 0


def test_full_size_hundred_iterations_keep_the_invariants(sphere):
    """100 iterations at the benchmark's size: surface particles stay on their
    owner facet (within the binary32 rounding of a point on a tilted plane),
    every particle stays inside the mesh (no particle past a facet plane of
    the sphere's hull, and within the facet sag of the unit sphere), no
    position is lost, and the projected force residual falls."""
    wl = sphere
    r = _relaxer(wl)
    r.step(count_pairs=False)
    a0 = r.by_id(r.accel)[:, :3].astype(np.float64)
    mov = wl.tag == synth.VOLUME
    R0 = np.sqrt(np.mean(np.sum(a0[mov] ** 2, 1)))
    for _ in range(99):
        r.step(keep_accel=False)
    r.build_cells()
    r.relax_step()
    a1 = r.by_id(r.accel)[:, :3].astype(np.float64)
    R1 = np.sqrt(np.mean(np.sum(a1[mov] ** 2, 1)))
    assert R1 < 0.5 * R0, (R0, R1)
    pos, owner, _, _ = r.host_state()
    assert np.all(np.isfinite(pos))
    mesh = wl.geoms[0].mesh
    s = np.nonzero(wl.tag == synth.SURFACE)[0]
    assert_on_facets(pos[s], mesh, owner[s], wl.geoms[0].dx)
    # the icosphere is convex: inside means below every facet plane; its
    # facets lie within the sag (< 3e-4) of the unit sphere
    rad = np.linalg.norm(pos.astype(np.float64), axis=1)
    assert rad.max() <= 1.0 + 1e-6
    v = np.nonzero(mov)[0]
    An, Bn, Cn = (mesh.vert[mesh.tri[:, q]] for q in range(3))
    fn = np.cross(Bn - An, Cn - An)
    fn /= np.linalg.norm(fn, axis=1, keepdims=True)
    off = np.einsum("ij,ij->i", fn, An)
    far = v[rad[v] > 1.0 - 1e-3]   # only particles within the sag band can reach a plane
    for c in range(0, len(far), 1000):
        sd = pos[far[c:c + 1000]].astype(np.float64) @ fn.T - off
        assert sd.max() < 0.0
    assert r.read_status() == 0
