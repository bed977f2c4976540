"""Gradient of the uniformity loss after K relaxation steps with respect to
the mesh vertices, on the GPU (an addition to the method of section 3.3).

The discrete decisions of each step (dt^2, owner facets before and after,
accepted or reverted moves, neighbour sets) are frozen at their forward
values; between them a step is smooth in the positions and in the facet
vertices (the map is written out in fppg.h above fppg_step_adjoint).

Reverse sweep with checkpointed recomputation:
  forward   K steps, keeping the state (pos, id, owner) every `checkpoint_every`
            steps (24 bytes per particle per checkpoint);
  loss      fppg_uniformity_loss on the final sorted state -> L, dL/dx;
  backward  per segment, last first: restore its checkpoint, recompute its
            steps storing per step the sorted state, cells, accelerations,
            owners after the step and the accept flags (about 45 bytes per
            particle per step), then walk the steps backwards:
              xbar_{n+1} (by id) -> sorted order of step n    fppg_vec_permute
              fppg_step_adjoint -> ybar (adjoint of a), xbar, facet-vertex terms
              xbar += J^T ybar                                   fppg_relax_hvp
              back to id order                                   fppg_vec_permute
  initial   singular points and the initial feature positions add their
            adjoints to their vertices: fppg_fixed_adjoint.
Checkpoints and per-step tapes include the feature table (segment and arc
length per slot), which the steps update in place.
All arithmetic runs in the library's kernels; this module marshals.
"""
from __future__ import annotations

import torch

from ._lib import S_FIXED_RANGE, check, ptr


def lattice_density(dx: float, h: float) -> float:
    """Rest density rho0 of the loss (fppg_lattice_density: the kernel sum of
    an infinite cubic lattice of spacing dx, computed by the library)."""
    import ctypes
    from . import _lib as L
    out = ctypes.c_double()
    check(L.lib().fppg_lattice_density(float(dx), float(h), ctypes.byref(out)))
    return float(out.value)


class _Tape:
    __slots__ = ("pos", "id", "owner", "cells", "accel", "amax", "owner_next", "accepted", "fseg", "fseg_next",
                 "fu_next")


def _restore(r, state):
    for dst, src in zip((r.pos, r.id, r.owner, r.feat_seg, r.feat_u), state):
        dst.copy_(src)


def _lib_call(r, name, *args):
    check(getattr(r.ctx.lib, name)(r.ctx.handle, *args), r.ctx.handle)


def uniformity_loss(r, rho0: float, grad: torch.Tensor | None = None) -> torch.Tensor:
    """(L, N) as a device double[2] at the relaxer's current sorted state
    (cells must be current); dL/dx into grad [N, 4] if given."""
    out = torch.zeros(2, dtype=torch.float64, device=r.dev)
    _lib_call(r, "fppg_uniformity_loss", r.geom.handle, r.n, ptr(r.pos), ptr(r.cell_start), r.move_mask,
              float(rho0), ptr(out), ptr(grad), r.ws_ptr, r.ws_bytes, r.stream)
    return out


class Tape:
    """What the reverse sweep needs from a forward run: the checkpoints, the
    final state, the loss and its gradient with respect to the final positions
    (by particle id)."""

    def __init__(self, K, every, ckpts, final, loss, xbar_id, feat0):
        self.K, self.every, self.ckpts, self.final = K, every, ckpts, final
        self.loss, self.xbar_id, self.feat0 = loss, xbar_id, feat0


def forward(r, K: int, rho0: float, checkpoint_every: int = 10) -> Tape:
    """K relaxation steps from the relaxer's state keeping checkpoints, then
    the uniformity loss of the final state and dL/dx (device, by id)."""
    if K < 0 or checkpoint_every < 1:
        raise ValueError("K >= 0 and checkpoint_every >= 1 required")
    if r.ws_bytes < 8 * (r.n + 2 * ((r.n + 255) // 256)) + 64:
        raise ValueError("workspace too small for the loss")
    ckpts = []
    feat0 = (r.feat_seg.clone(), r.feat_u.clone())
    for step in range(K):
        if step % checkpoint_every == 0:
            ckpts.append((step, r.pos.clone(), r.id.clone(), r.owner.clone(), r.feat_seg.clone(), r.feat_u.clone()))
        r.step(keep_accel=False)
    final = (r.pos.clone(), r.id.clone(), r.owner.clone(), r.feat_seg.clone(), r.feat_u.clone())
    r.build_cells()
    g = torch.zeros((r.n, 4), dtype=torch.float32, device=r.dev)
    out = uniformity_loss(r, rho0, g)
    xbar_id = torch.zeros_like(g)
    _lib_call(r, "fppg_vec_permute", r.n, ptr(g), ptr(r.id), 1, ptr(xbar_id), r.stream)
    return Tape(K, checkpoint_every, ckpts, final, out, xbar_id, feat0)


def backward(r, tape: Tape, n_vert: int | None = None) -> torch.Tensor:
    """Reverse sweep of a forward run: dL/dV [n_vert, 3] (device, float64).
    The relaxer is left in the state after the K steps."""
    dev, n = r.dev, r.n
    n_vert = int(n_vert if n_vert is not None else r.n_vert)
    xbar_id = tape.xbar_id.clone()
    vbar = torch.zeros(3 * n_vert, dtype=torch.int64, device=dev)
    xb_next = torch.empty_like(xbar_id)
    xb = torch.empty_like(xbar_id)
    yb = torch.empty_like(xbar_id)
    jt = torch.empty_like(xbar_id)
    first = None
    ckpts = tape.ckpts
    for ci in range(len(ckpts) - 1, -1, -1):
        s0, pos, ids, own, fseg, fu = ckpts[ci]
        s1 = ckpts[ci + 1][0] if ci + 1 < len(ckpts) else tape.K
        _restore(r, (pos, ids, own, fseg, fu))
        tapes = []
        for _ in range(s0, s1):
            t = _Tape()
            r.build_cells()
            t.pos, t.id, t.owner, t.cells = r.pos.clone(), r.id.clone(), r.owner.clone(), r.cell_start.clone()
            t.fseg = r.feat_seg.clone()
            r.relax_step(keep_accel=True)
            t.accel, t.amax = r.accel.clone(), r.amax.clone()
            t.accepted = torch.empty(n, dtype=torch.uint8, device=dev)
            r.project_record(t.accepted)
            t.owner_next = r.owner.clone()
            t.fseg_next, t.fu_next = r.feat_seg.clone(), r.feat_u.clone()
            tapes.append(t)
        for t in reversed(tapes):
            _lib_call(r, "fppg_vec_permute", n, ptr(xbar_id), ptr(t.id), 0, ptr(xb_next), r.stream)
            _lib_call(r, "fppg_step_adjoint", r.geom.handle, n, ptr(t.pos), ptr(t.accepted), ptr(t.owner),
                      ptr(t.owner_next), ptr(t.accel), ptr(t.amax), ptr(t.fseg), ptr(t.fseg_next), ptr(t.fu_next),
                      r.n_feat, r.move_mask, ptr(xb_next), ptr(yb), ptr(xb), ptr(vbar), r.stream)
            _lib_call(r, "fppg_relax_hvp", r.geom.handle, n, ptr(t.pos), ptr(t.cells), r.move_mask, 1,
                      ptr(yb), ptr(jt), r.stream)
            r.axpby(1.0, jt, 1.0, xb)
            _lib_call(r, "fppg_vec_permute", n, ptr(xb), ptr(t.id), 1, ptr(xbar_id), r.stream)
        if ci == 0 and tapes:
            first = tapes[0]
    # particles that do not move depend on the vertices directly
    if first is not None:
        pos0, own0, ids0 = first.pos, first.owner, first.id
    else:
        _restore(r, tape.final)
        r.build_cells()
        pos0, own0, ids0 = r.pos, r.owner, r.id
    _lib_call(r, "fppg_vec_permute", n, ptr(xbar_id), ptr(ids0), 0, ptr(xb), r.stream)
    _lib_call(r, "fppg_fixed_adjoint", r.geom.handle, n, ptr(pos0), ptr(own0), ptr(tape.feat0[0]),
              ptr(tape.feat0[1]), r.n_feat, r.move_mask, ptr(xb), ptr(vbar), r.stream)
    vd = torch.empty(3 * n_vert, dtype=torch.float64, device=dev)
    _lib_call(r, "fppg_fixed_to_double", 3 * n_vert, ptr(vbar), ptr(vd), r.stream)
    # the device status is read (and cleared) here: a vertex gradient outside
    # the fixed-point range is an error, not a value
    if r.read_status() & S_FIXED_RANGE:
        raise FloatingPointError("a vertex gradient left the fixed-point range |g| < 2^23")
    _restore(r, tape.final)
    return vd.view(n_vert, 3)


def mesh_gradient(r, K: int, rho0: float, checkpoint_every: int = 10, n_vert: int | None = None):
    """Run K relaxation steps from the relaxer's state and return
    (L, dL/dV [n_vert, 3] float64 numpy) with V the batch's mesh vertices in
    global numbering. The relaxer ends in the state after the K steps."""
    tape = forward(r, K, rho0, checkpoint_every)
    g = backward(r, tape, n_vert)
    torch.cuda.synchronize(r.dev)
    return float(tape.loss[0].item()), g.cpu().numpy()


class RelaxedUniformity(torch.autograd.Function):
    """L(V): the uniformity loss after K relaxation steps of the relaxer's
    particles on the mesh with vertices V, as a differentiable torch function.
    The geometry is the one the relaxer was built with, so V must hold those
    vertices (checked); forward runs the steps keeping checkpoints, backward
    runs the reverse sweep in the library's kernels.

        L = RelaxedUniformity.apply(V, relaxer, K, rho0, checkpoint_every)
        L.backward()      # V.grad = dL/dV
    """

    @staticmethod
    def forward(ctx, V, r, K, rho0, checkpoint_every=10):
        want = torch.as_tensor(r.vert, dtype=torch.float64)
        if V.shape != want.shape or not torch.equal(V.detach().to("cpu", torch.float64), want):
            raise ValueError("V must be the vertices the relaxer's geometry was built from")
        tape = forward(r, int(K), float(rho0), int(checkpoint_every))
        ctx.r, ctx.tape = r, tape
        return tape.loss[0].to(V.device, V.dtype)

    @staticmethod
    def backward(ctx, gL):
        g = backward(ctx.r, ctx.tape)
        ctx.r = ctx.tape = None
        return (gL * g.to(gL.device, gL.dtype)).to(gL.dtype), None, None, None, None
