"""Pins of the multi-resolution oracle (oracle/multires.py) by its reductions
and invariants:

  * all levels 0: the single-resolution force and step, bit for bit
  * two particles of levels 0 and 1: the closed form K(h_ij)(1 - r/2h_ij)^3 r,
    and no force once r >= h_i + h_j although r < 2h
  * every pair term is antisymmetric (h_ij, the predicate and K symmetric):
    the accelerations of an all-moving volume cloud sum to zero
  * halving every length: a configuration at level 1 is the level-0 one scaled
    by 1/2, with the same neighbours and 16 times the accelerations (a ~ h^-4)
  * the time step moves the fastest particle, measured in its own h_i, by
    exactly h_i / 16, and no particle farther
"""
import numpy as np
import pytest

import synth
from oracle import force as F
from oracle import multires as MR
from oracle import step as S
from oracle.kernel import force_coef
from synth import meshes as M


def _cloud(n=400, seed=3, scale=0.4, h=0.1):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(-scale, scale, size=(n, 3))
    wl = synth.workload.custom_workload(M.cube((-1, -1, -1), (1, 1, 1)), h / 1.3, pos, np.full(n, 3, np.int32))
    return wl


def test_all_levels_zero_is_the_single_resolution_step():
    wl = synth.sphere_workload(level=2, dx=0.15, seed=4)
    lev = np.zeros(wl.n, np.int64)
    a0, S0, c0 = F.accel(wl)
    a1, S1, c1 = MR.accel(wl, lev)
    assert np.array_equal(c0, c1)
    assert np.array_equal(a0, a1) and np.array_equal(S0, S1)
    r0 = S.relax_step(wl)
    r1 = MR.relax_step(wl, lev)
    assert np.array_equal(r0.pos32, r1.pos32) and np.array_equal(r0.reverted, r1.reverted)


def test_two_particles_of_different_levels():
    h = float(np.float32(0.1))
    for r in (0.03, 0.1, 0.14, 0.1499, 0.16, 0.19):
        pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        wl = synth.workload.custom_workload(M.cube((-1, -1, -1), (1, 1, 1)), h / 1.3, pos, np.full(2, 3, np.int32))
        lev = np.array([0, 1])
        a, _, cnt = MR.accel(wl, lev)
        hs = np.float32(wl.geoms[0].h) + np.float32(wl.geoms[0].h) * np.float32(0.5)
        rr = float(np.float64(np.float32(r)))
        if rr * rr < float(np.float32(hs) * np.float32(hs)):
            h32 = float(wl.geoms[0].h)
            hij = 0.5 * (h32 + 0.5 * h32)          # exact in FP64
            want = force_coef(hij) * (1 - rr / (2 * hij)) ** 3 * rr
            assert cnt[0] == 1 and a[0, 0] == pytest.approx(-want, rel=1e-14)
            assert a[1, 0] == pytest.approx(want, rel=1e-14)
        else:
            assert cnt[0] == 0 and np.all(a == 0.0)


def test_pair_terms_are_antisymmetric():
    wl = _cloud(n=800)
    rng = np.random.Generator(np.random.PCG64(7))
    lev = rng.integers(0, 4, wl.n)
    a, Ssum, cnt = MR.accel(wl, lev)
    assert cnt.sum() > 4000
    assert np.abs(a.sum(0)).max() <= 1e-10 * Ssum.sum()


def test_halving_every_length_scales_the_force_by_sixteen():
    wl0 = _cloud(n=300, seed=5)
    wl1 = _cloud(n=300, seed=5)
    wl1.pos = (wl0.pos * np.float32(0.5)).astype(np.float32)
    a0, S0, c0 = MR.accel(wl0, np.zeros(wl0.n, np.int64))
    a1, S1, c1 = MR.accel(wl1, np.ones(wl1.n, np.int64))
    assert np.array_equal(c0, c1)
    np.testing.assert_allclose(a1, 16.0 * a0, rtol=1e-13, atol=1e-13 * np.abs(a0).max())


def test_time_step_moves_each_particle_at_most_its_h_over_16():
    wl = synth.workload.multires_sphere_workload(level=2, dx=0.2)
    out = MR.relax_step(wl, wl.level)
    h = MR.h_of(wl.geoms[0], wl.level).astype(np.float64)
    ratio = np.linalg.norm(out.tau[wl.gid][:, None] * out.a, axis=1) / h
    mov = F.moving_mask(wl.tag, wl.move_mask)
    assert ratio[mov].max() == pytest.approx(1.0 / 16.0, rel=1e-12)
    assert np.all(ratio[mov] <= 1.0 / 16.0 * (1 + 1e-12))
