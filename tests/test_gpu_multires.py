"""GPU parity of the multi-resolution relaxation (per-particle levels,
h_ij = (h_i + h_j)/2) against oracle/multires.py: neighbour counts bit-exact,
forces within 1e-5 S_i, one step's positions within 1e-5 of the FP64 step,
the time step rule, and the refusal of the sweeps that take one length."""
import numpy as np
import pytest

import synth
from oracle import force as oforce
from oracle import multires as omr
from synth import meshes as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _relaxer(wl):
    from paper_2501_03056_amd import Relaxer
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Relaxer(wl, device=0)


def _random_levels():
    """A cube of volume particles with random levels 0..3 (every pair kind)."""
    rng = np.random.Generator(np.random.PCG64(9))
    dx = 0.1
    pos = rng.uniform(0.05, 0.95, size=(3000, 3))
    wl = synth.workload.custom_workload(M.cube(), dx, pos, np.full(len(pos), synth.VOLUME, np.int32))
    wl.geoms[0].max_level = 3
    wl.level = rng.integers(0, 4, wl.n).astype(np.int32)
    return wl


CASES = {
    "mr_sphere": lambda: synth.workload.multires_sphere_workload(level=3, dx=0.12),
    "random_levels": _random_levels,
}


@pytest.mark.parametrize("case", list(CASES))
def test_forces_and_counts_match_the_oracle(case):
    wl = CASES[case]()
    print(f"[multires] {case} n={wl.n} levels={np.bincount(wl.level)}", flush=True)
    r = _relaxer(wl)
    r.build_cells()
    r.relax_step(count_pairs=True)
    acc = r.by_id(r.accel)
    a64, S, cnt = omr.accel(wl, wl.level)
    mov = oforce.moving_mask(wl.tag, wl.move_mask)
    assert np.array_equal(acc[:, 3].astype(np.int64), np.where(mov, cnt, 0))
    err = np.linalg.norm(acc[:, :3].astype(np.float64) - a64, axis=1)
    assert np.all(err[mov] <= 1e-5 * S[mov]), float(np.max(err[mov] / np.maximum(S[mov], 1e-300)))
    amax = omr.amax_per_geometry(wl, a64, wl.level)
    assert np.allclose(r.amax.cpu().numpy(), amax, rtol=1e-5)
    assert r.read_status() == 0


def test_one_step_matches_the_oracle():
    wl = CASES["mr_sphere"]()
    r = _relaxer(wl)
    r.step()
    ref = omr.relax_step(wl, wl.level)
    pos, owner, _, _ = r.host_state()
    ok = ~ref.margin
    x = ref.pos32.astype(np.float64)
    tol = 1e-5 * np.maximum(np.abs(x).max(1), wl.geoms[0].dx)
    err = np.abs(pos.astype(np.float64) - x).max(1)
    assert not (ok & (err > tol)).any(), float(err[ok].max())
    s = ok & (wl.tag == synth.SURFACE)
    assert np.array_equal(owner[s], ref.owner[s])
    # every particle moved at most its own h_i / 16
    h = omr.h_of(wl.geoms[0], wl.level).astype(np.float64)
    moved = np.linalg.norm(pos.astype(np.float64) - wl.pos.astype(np.float64), axis=1)
    vol = wl.tag == synth.VOLUME
    assert np.all(moved[vol] <= h[vol] / 16.0 * (1 + 1e-5) + 1e-7)


def test_levels_zero_match_the_single_resolution_kernel():
    """max_level > 0 with every particle at level 0: the level-aware kernel
    gives the single-resolution forces (to FP32 rounding)."""
    wl = synth.sphere_workload(level=3, dx=0.08, seed=2)
    r0 = _relaxer(wl)
    r0.build_cells()
    r0.relax_step()
    a0 = r0.by_id(r0.accel)[:, :3]
    wl.geoms[0].max_level = 1
    wl.level = np.zeros(wl.n, np.int32)
    r1 = _relaxer(wl)
    r1.build_cells()
    r1.relax_step()
    a1 = r1.by_id(r1.accel)[:, :3]
    _, S, _ = oforce.accel(wl)
    err = np.linalg.norm(a1.astype(np.float64) - a0, axis=1)
    assert np.all(err <= 2e-6 * np.maximum(S, 1e-30))


def test_sweeps_with_one_length_refuse_a_multiresolution_geometry():
    from paper_2501_03056_amd._lib import E_UNSUPPORTED, FppgError
    wl = CASES["mr_sphere"]()
    r = _relaxer(wl)
    r.build_cells()
    v = torch.zeros_like(r.pos)
    with pytest.raises(FppgError) as e:
        r.hvp(v)
    assert e.value.status == E_UNSUPPORTED
