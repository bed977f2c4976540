"""Pins of the mesh-gradient oracle (oracle/grad.py) on the CPU.

The gradient is not in the paper; its definition (frozen decisions, smooth
map between them) is pinned three ways:
  * the replayed smooth map reproduces the oracle's own forward steps
    (step.relax_step, which projects with its own closest-point search);
  * the replayed loss equals metrics.uniformity_loss on the same positions;
  * autograd through the replay agrees with central differences.
"""
import numpy as np
import pytest
import torch

import synth.meshes as M
import synth.workload as W
from oracle import grad as G
from oracle import metrics

SURF_VOL = (1 << W.SURFACE) | (1 << W.VOLUME)


@pytest.fixture(scope="module")
def tetra():
    wl = W.tetra_workload(dx=0.12, move_mask=SURF_VOL)
    rec = G.record(wl, 3)
    return wl, rec


def test_singular_owner_is_its_vertex(tetra):
    wl, _ = tetra
    s = wl.tag == W.SINGULAR
    assert s.sum() == 4
    np.testing.assert_array_equal(wl.pos[s], wl.geoms[0].mesh.vert[wl.owner[s]].astype(np.float32))


def test_feature_ends_are_mesh_vertices(tetra):
    wl, _ = tetra
    lines = wl.geoms[0].mesh.lines
    V = wl.geoms[0].mesh.vert
    p = lines.seg_p.reshape(-1, 2, 3)
    np.testing.assert_allclose(p[:, 0], V[lines.seg_vert[:, 0]], atol=1e-15)
    np.testing.assert_allclose(p[:, 1], V[lines.seg_vert[:, 1]], atol=1e-15)


def test_fixed_positions_match_the_workload(tetra):
    wl, _ = tetra
    V = torch.as_tensor(wl.geoms[0].mesh.vert)
    x = G.fixed_positions(wl, V).numpy()
    fixed = (wl.tag == W.SINGULAR) | (wl.tag == W.FEATURE)
    np.testing.assert_allclose(x[fixed], wl.pos[fixed].astype(np.float64), atol=2e-7)


def test_replay_reproduces_the_recorded_forward(tetra):
    wl, rec = tetra
    V = torch.as_tensor(wl.geoms[0].mesh.vert)
    assert any(a.any() for a in rec.accepted)
    for K in range(1, len(rec.tau) + 1):
        sub = G.Record(rec.pos32[:K + 1], rec.owner[:K + 1], rec.tau[:K], rec.accepted[:K], rec.pairs[:K], None)
        x = G.replay(wl, V, sub).numpy()
        np.testing.assert_allclose(x, rec.pos32[K].astype(np.float64), rtol=0, atol=2e-6 * K)


def test_replay_surface_particles_stay_on_their_facets(tetra):
    wl, rec = tetra
    V = torch.as_tensor(wl.geoms[0].mesh.vert)
    x = G.replay(wl, V, rec).numpy()
    mesh = wl.geoms[0].mesh
    s = np.nonzero(wl.tag == W.SURFACE)[0]
    own = rec.owner[-1][s]
    A, B, C = (mesh.vert[mesh.tri[own, c]] for c in range(3))
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    np.testing.assert_allclose(np.einsum("ij,ij->i", x[s] - A, n), 0.0, atol=1e-12)


def test_replayed_loss_matches_metrics(tetra):
    wl, rec = tetra
    x = rec.pos32[-1]
    L = float(G.loss(wl, torch.as_tensor(x.astype(np.float64)), rec))
    assert L == pytest.approx(metrics.uniformity_loss(wl, pos32=x), rel=1e-12)


def test_mesh_gradient_matches_central_differences(tetra):
    wl, rec = tetra
    L, g = G.mesh_gradient(wl, rec)
    fd = G.mesh_gradient_fd(wl, rec, eps=1e-6)
    assert np.abs(g).max() > 1e-3
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-6 * np.abs(g).max() + 1e-9)


def test_mesh_gradient_is_consistent_with_rigid_motions():
    """Moving the mesh and every particle rigidly leaves the loss unchanged, so
    the vertex gradient plus the initial-position gradient has zero net force
    (translations) and zero net torque (rotations, which turn the normals)."""
    wl = W.tetra_workload(dx=0.14, move_mask=SURF_VOL)
    rec = G.record(wl, 2)
    V = torch.as_tensor(wl.geoms[0].mesh.vert.copy()).requires_grad_(True)
    mov = torch.as_tensor((wl.tag == W.SURFACE) | (wl.tag == W.VOLUME))
    x0 = torch.as_tensor(wl.pos.astype(np.float64)).requires_grad_(True)
    L = G.loss(wl, G.replay(wl, V, rec, x0=x0), rec)
    gV, gx = torch.autograd.grad(L, (V, x0))
    scale = float(torch.linalg.norm(gV))
    assert scale > 1e-3
    force = gV.sum(0) + gx[mov].sum(0)
    torque = torch.cross(V.detach(), gV, dim=1).sum(0) + torch.cross(x0.detach()[mov], gx[mov], dim=1).sum(0)
    assert float(torch.linalg.norm(force)) <= 1e-9 * scale
    assert float(torch.linalg.norm(torque)) <= 1e-9 * scale


@pytest.fixture(scope="module")
def cylinder():
    """Cylinder with every class moving: feature particles walk along the two
    24-segment rim loops and some cross segment ends."""
    wl = W.cylinder_workload(dx=0.08)
    rec = G.record(wl, 6)
    return wl, rec


def test_feature_walks_cross_segments(cylinder):
    wl, rec = cylinder
    fs = np.array(rec.feat_seg)
    assert (fs[1:] != fs[:-1]).any()
    f = wl.tag == W.FEATURE
    assert all(a[f].any() for a in rec.accepted)


def test_replay_with_moving_features_reproduces_the_forward(cylinder):
    wl, rec = cylinder
    V = torch.as_tensor(wl.geoms[0].mesh.vert)
    x = G.replay(wl, V, rec).numpy()
    np.testing.assert_allclose(x, rec.pos32[-1].astype(np.float64), rtol=0, atol=1e-6)


def test_mesh_gradient_with_moving_features_matches_central_differences(cylinder):
    wl, rec = cylinder
    _, g = G.mesh_gradient(wl, rec)
    rows = list(range(0, len(wl.geoms[0].mesh.vert), 5))
    fd = G.mesh_gradient_fd(wl, rec, eps=1e-6, verts=rows)
    assert np.abs(g[rows]).max() > 1e-3
    np.testing.assert_allclose(g[rows], fd[rows], rtol=0, atol=1e-6 * np.abs(g).max())
