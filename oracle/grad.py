"""Gradient of the uniformity loss with respect to mesh vertices through K
relaxation steps (FP64, torch autograd). Not in the paper: an addition that
differentiates the relaxation of section 3.3.

Reading (parity unpinned as a definition; its pins are below): the discrete
decisions of every step are frozen at their forward values: the time step
dt_n^2 (Eq. 22-23 reading), each particle's owner facet (feature segment)
before and after the step, whether its move was accepted or reverted, the
direction of a feature particle's walk, and the neighbour pairs. Between
decisions the step is a smooth map of the positions and of the mesh:

    y = x + dt^2 P_o a(x)                 P_o = I - n_o n_o^T for surface, I for volume
    x' = y - ((y - A_t) . n_t) n_t        accepted surface move onto facet t
    x' = y                                accepted volume move
    u' = u + dt^2 a(x).t_s + c            accepted feature move from segment s to s':
    x' = P0_s' + u' t_s'                  c = -(lengths of the segments walked off
                                          forwards) + (lengths of those walked onto
                                          backwards), t = (P1 - P0)/|P1 - P0|
    x' = x                                reverted move, or a particle that does not move

with n = (B - A) x (C - A) / |.| of the facet's vertices and (s, u) a feature
particle's segment and arc length. Particles that do not move are functions of
the mesh: a singular particle sits on its vertex, a feature particle at arc
length u of its segment. Feature particles start on the mesh (at their
initial (s, u)); surface and volume particles start at their given positions.
The loss is metrics.uniformity_loss of the final positions.

`record` runs the oracle's own forward (step.relax_step) and stores the
decisions; `replay` re-evaluates the K steps in torch from the vertex array
V; `mesh_gradient` returns dL/dV by autograd. Pins (tests): replay(V) matches
the recorded forward (which projects with its own closest-point search), the
replayed loss equals metrics.uniformity_loss, autograd matches central
differences of replay, and the gradient has zero net force and torque under
rigid motions of mesh and particles together.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import force as F
from . import step as S
from .kernel import alpha as kalpha
from .metrics import lattice_density
from .neighbors import pair_d2, rc2_f32

SINGULAR, FEATURE, SURFACE, VOLUME = 0, 1, 2, 3


def _pairs(wl, pos32, receivers_mask, with_rank=True):
    """(I, J) pairs passing the binary32 predicate, receivers in the mask; the
    class rule applied when with_rank."""
    I, J = [], []
    members = np.arange(wl.n)
    rc2 = rc2_f32(wl.geoms[0].h)
    rank = F.RANK[wl.tag]
    rec = np.nonzero(receivers_mask)[0]
    step = max(1, (1 << 24) // max(wl.n, 1))
    for s in range(0, len(rec), step):
        r = rec[s:s + step]
        hit = pair_d2(pos32[r][:, None, :], pos32[None, :, :]) < rc2
        hit &= members[None, :] != r[:, None]
        if with_rank:
            hit &= rank[None, :] <= rank[r][:, None]
        b, m = np.nonzero(hit)
        I.append(r[b])
        J.append(m)
    return np.concatenate(I), np.concatenate(J)


@dataclass
class Record:
    pos32: list          # binary32 state entering each step, [K+1] (last = final state)
    owner: list          # owner before each step, [K+1]
    tau: list            # dt^2 of each step
    accepted: list       # bool [N] per step: the move was applied
    pairs: list          # force pairs (I, J) per step
    loss_pairs: tuple    # density pairs of the final state
    feat_seg: list = None   # feature segment per slot before each step, [K+1]
    feat_u: list = None     # feature arc length per slot before each step, [K+1]
    du: list = None         # feature arc-length increment per particle per step


def record(wl, K: int) -> Record:
    """K oracle steps from the workload's state (single geometry)."""
    assert len(wl.geoms) == 1, "single geometry"
    mov = F.moving_mask(wl.tag, wl.move_mask)
    pos, owner = wl.pos.copy(), wl.owner.copy()
    fs, fu = wl.feat_seg.copy(), wl.feat_u.copy()
    rec = Record([pos], [owner], [], [], [], None, [fs], [fu], [])
    for _ in range(K):
        out = S.relax_step(wl, pos32=pos, owner=owner, feat_seg=fs, feat_u=fu)
        rec.tau.append(float(out.tau[0]))
        rec.accepted.append(mov & ~out.reverted)
        rec.pairs.append(_pairs(wl, pos, mov))
        rec.du.append(out.du.copy())
        pos, owner, fs, fu = out.pos32, out.owner, out.feat_seg, out.feat_u
        rec.pos32.append(pos)
        rec.owner.append(owner)
        rec.feat_seg.append(fs)
        rec.feat_u.append(fu)
    rec.loss_pairs = _pairs(wl, pos, mov, with_rank=False)
    return rec


def _frames(V, tri):
    A, B, C = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    n = torch.cross(B - A, C - A, dim=1)
    return A, n / torch.linalg.norm(n, dim=1, keepdim=True)


def _segments(wl, V):
    """P0, unit tangent and length of every feature segment, from V."""
    sv = torch.as_tensor(wl.geoms[0].mesh.lines.seg_vert.astype(np.int64))
    P0, P1 = V[sv[:, 0]], V[sv[:, 1]]
    L = torch.linalg.norm(P1 - P0, dim=1)
    return P0, (P1 - P0) / L[:, None], L


def _walk(lines, s, s2, forward):
    """Segments a feature particle walks off (forwards) or onto (backwards)
    going from segment s to s2 along its line."""
    lsb = lines.line_seg_begin
    line = int(np.searchsorted(lsb, s, side="right") - 1)
    lo, hi, closed = int(lsb[line]), int(lsb[line + 1]), bool(lines.line_closed[line])
    out, k = [], int(s)
    while k != s2:
        if forward:
            out.append(k)
            k = k + 1 if k + 1 < hi else (lo if closed else None)
        else:
            k = k - 1 if k > lo else (hi - 1 if closed else None)
            out.append(k)
        assert k is not None and len(out) <= hi - lo, "feature walk left its line"
    return out


def fixed_positions(wl, V):
    """Positions of the particles that do not move, as functions of V (all
    feature particles: their initial positions)."""
    geo = wl.geoms[0]
    x = torch.as_tensor(wl.pos.astype(np.float64)).clone()
    sing = np.nonzero(wl.tag == SINGULAR)[0]
    if len(sing):
        x[sing] = V[torch.as_tensor(wl.owner[sing].astype(np.int64))]
    feat = np.nonzero(wl.tag == FEATURE)[0]
    if len(feat):
        sv = geo.mesh.lines.seg_vert
        slots = wl.owner[feat]
        seg = wl.feat_seg[slots]
        P0 = V[torch.as_tensor(sv[seg, 0].astype(np.int64))]
        P1 = V[torch.as_tensor(sv[seg, 1].astype(np.int64))]
        D = P1 - P0
        u = torch.as_tensor(wl.feat_u[slots])
        x[feat] = P0 + (u / torch.linalg.norm(D, dim=1))[:, None] * D
    return x


def replay(wl, V, rec: Record, x0=None):
    """The K recorded steps re-evaluated in FP64 from the vertices V."""
    geo = wl.geoms[0]
    h = float(geo.h)
    Kc = 5.0 * kalpha(h) / (h * h)
    tri = torch.as_tensor(geo.mesh.tri.astype(np.int64))
    A, nrm = _frames(V, tri)
    mov = torch.as_tensor(F.moving_mask(wl.tag, wl.move_mask))
    surf = torch.as_tensor(wl.tag == SURFACE)
    x = fixed_positions(wl, V)
    if x0 is not None:
        x = torch.where(mov[:, None] & (torch.as_tensor(wl.tag) != FEATURE)[:, None], x0, x)
    fmov = np.nonzero(F.moving_mask(wl.tag, wl.move_mask) & (wl.tag == FEATURE))[0]
    if len(fmov):
        P0, T, L = _segments(wl, V)
        lines = geo.mesh.lines
        u = torch.as_tensor(wl.feat_u.copy())               # arc length per slot (state)
    for n in range(len(rec.tau)):
        I = torch.as_tensor(rec.pairs[n][0].astype(np.int64))
        J = torch.as_tensor(rec.pairs[n][1].astype(np.int64))
        r = x[I] - x[J]
        t = torch.clamp(1.0 - torch.linalg.norm(r, dim=1) / (2.0 * h), min=0.0)
        a = torch.zeros_like(x).index_add(0, I, Kc * t[:, None] ** 3 * r)
        own_o = torch.as_tensor(np.where(wl.tag == SURFACE, rec.owner[n], 0).astype(np.int64))
        no = nrm[own_o]
        a_t = torch.where(surf[:, None], a - (a * no).sum(1, keepdim=True) * no, a)
        y = x + rec.tau[n] * a_t
        own_t = torch.as_tensor(np.where(wl.tag == SURFACE, rec.owner[n + 1], 0).astype(np.int64))
        nt, At = nrm[own_t], A[own_t]
        proj = y - ((y - At) * nt).sum(1, keepdim=True) * nt
        moved = torch.where(surf[:, None], proj, y)
        if len(fmov):
            rows, vals, slots, us = [], [], [], []
            for i in fmov:
                if not rec.accepted[n][i]:
                    continue
                slot = int(wl.owner[i])
                s0, s2 = int(rec.feat_seg[n][slot]), int(rec.feat_seg[n + 1][slot])
                du = rec.tau[n] * (a[i] * T[s0]).sum()
                c = 0.0
                for k in _walk(lines, s0, s2, rec.du[n][i] > 0):
                    c = c + (-L[k] if rec.du[n][i] > 0 else L[k])
                un = u[slot] + du + c
                rows.append(int(i))
                vals.append(P0[s2] + un * T[s2])
                slots.append(slot)
                us.append(un)
            if rows:
                u = u.index_put((torch.as_tensor(slots),), torch.stack(us))
                moved = moved.index_copy(0, torch.as_tensor(rows), torch.stack(vals))
        acc = torch.as_tensor(rec.accepted[n])
        x = torch.where(acc[:, None], moved, x)
    return x


def loss(wl, x, rec: Record):
    """Uniformity loss (metrics.uniformity_loss) of positions x over the recorded pairs."""
    geo = wl.geoms[0]
    h = float(geo.h)
    al = kalpha(h)
    I = torch.as_tensor(rec.loss_pairs[0].astype(np.int64))
    J = torch.as_tensor(rec.loss_pairs[1].astype(np.int64))
    q = torch.linalg.norm(x[I] - x[J], dim=1) / h
    t = torch.clamp(1.0 - 0.5 * q, min=0.0)
    w = al * t ** 4 * (2.0 * q + 1.0)
    rho = torch.full((wl.n,), al, dtype=torch.float64).index_add(0, I, w)
    mov = torch.as_tensor(F.moving_mask(wl.tag, wl.move_mask))
    rho0 = lattice_density(geo.dx, h)
    return torch.mean((rho[mov] / rho0 - 1.0) ** 2)


def mesh_gradient(wl, rec: Record):
    """(L, dL/dV) by autograd through the replayed steps."""
    V = torch.as_tensor(wl.geoms[0].mesh.vert.copy()).requires_grad_(True)
    L = loss(wl, replay(wl, V, rec), rec)
    (g,) = torch.autograd.grad(L, V)
    return float(L.detach()), g.numpy()


def mesh_gradient_fd(wl, rec: Record, eps=1e-6, verts=None):
    """Central differences of replay + loss in the coordinates of the given
    vertices (default: all); other rows are left 0."""
    V0 = wl.geoms[0].mesh.vert.copy()
    g = np.zeros_like(V0)
    with torch.no_grad():
        for v in (range(V0.shape[0]) if verts is None else verts):
            for c in range(3):
                Vp, Vm = V0.copy(), V0.copy()
                Vp[v, c] += eps
                Vm[v, c] -= eps
                lp = float(loss(wl, replay(wl, torch.as_tensor(Vp), rec), rec))
                lm = float(loss(wl, replay(wl, torch.as_tensor(Vm), rec), rec))
                g[v, c] = (lp - lm) / (2 * eps)
    return g
