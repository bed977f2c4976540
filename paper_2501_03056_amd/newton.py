"""Newton-Krylov relaxation on one GPU.

The plain loop of Algorithm 1 moves every particle by dt^2 a with
dt^2 = (h/16)/max|a|: the fastest particle always moves h/16, so the loop
settles into a noise floor of the force residual instead of converging.
Relaxation is done when the tangential forces vanish,

    F(x) = P a(x) = 0,

and Newton's method solves that system directly:

    solve  (P J P) d = -F  with MINRES            -P J v in one sweep from
                                                   fppg_relax_hvp_projected
    cap every particle's move at move_cap * h    fppg_vec_clamp
    x <- Pi(x + s d), s = 1, 1/2, ... until |F|^2 decreases   fppg_displace + fppg_project

For one moving class with fixed other sources J = -Hess(E) is symmetric but
indefinite (pair curvature across a bond is negative), which is exactly the
case MINRES handles (conjugate gradients would break down on it). Every
vector operation runs in the library's kernels; this module only sequences
them and reads back scalars.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import torch

from .relax import Relaxer


def projected_force(r: Relaxer) -> torch.Tensor:
    """Rebuild the cells at the current positions and return F = P a."""
    r.build_cells()
    r.relax_step(keep_accel=True, forces_only=True)
    b = r.accel.clone()
    r.tangent(b)
    return b


def force_residual(r: Relaxer, b: torch.Tensor, n_moving: int) -> float:
    """sqrt(mean over moving particles of |P a|^2)."""
    return math.sqrt(max(r.dot(b, b), 0.0) / max(n_moving, 1))


@dataclass
class NewtonLog:
    residual: list = field(default_factory=list)   # (wall s, R) after every accepted step
    newton_iters: int = 0
    krylov_iters: int = 0
    backtracks: int = 0
    checkpoint: tuple | None = None                  # device snapshot (Relaxer.snapshot)


class _Minres:
    """MINRES (Paige-Saunders) for A x = b with A = -P J P, on device vectors.
    One iteration: the operator in one sweep (fppg_relax_hvp_projected), two
    axpbys, two dot products, one fused direction + iterate update
    (fppg_vec_combine3); the Lanczos vectors rotate through three buffers."""

    def __init__(self, r: Relaxer, like: torch.Tensor):
        self.r = r
        self.v, self.y, self.r1, self.r2 = (torch.empty_like(like) for _ in range(4))
        self.w, self.w1, self.w2 = (torch.empty_like(like) for _ in range(3))

    def solve(self, b: torch.Tensor, x: torch.Tensor, rtol: float, maxit: int) -> int:
        r = self.r
        x.zero_()
        beta1 = math.sqrt(max(r.dot(b, b), 0.0))
        if beta1 == 0.0:
            return 0
        self.r1.copy_(b)
        self.r2.copy_(b)
        oldb, beta, dbar, epsln, phibar, cs, sn = 0.0, beta1, 0.0, 0.0, beta1, -1.0, 0.0
        self.w.zero_()
        self.w2.zero_()
        it = 0
        for it in range(1, maxit + 1):
            r.axpby(1.0 / beta, self.r2, 0.0, self.v)           # v = y / beta (r2 holds y)
            r.hvp_projected(self.v, -1.0, self.y)               # y = A v
            if it >= 2:
                r.axpby(-beta / oldb, self.r1, 1.0, self.y)
            alfa = r.dot(self.v, self.y)
            r.axpby(-alfa / beta, self.r2, 1.0, self.y)
            # (r1, r2) <- (r2, y); the old r1 buffer becomes the next y
            self.r1, self.r2, self.y = self.r2, self.y, self.r1
            oldb, beta = beta, math.sqrt(max(r.dot(self.r2, self.r2), 0.0))
            oldeps = epsln
            delta = cs * dbar + sn * alfa
            gbar = sn * dbar - cs * alfa
            epsln = sn * beta
            dbar = -cs * beta
            gamma = max(math.hypot(gbar, beta), 1e-300)
            cs, sn = gbar / gamma, beta / gamma
            phi = cs * phibar
            phibar = sn * phibar
            # w_new = (v - oldeps w1 - delta w2) / gamma with (w1, w2) <- (w2, w); x += phi w_new
            self.w1, self.w2, self.w = self.w2, self.w, self.w1
            r.combine3(1.0 / gamma, self.v, -oldeps / gamma, self.w1, -delta / gamma, self.w2, self.w, phi, x)
            if phibar <= rtol * beta1 or beta == 0.0:
                break
        return it


def newton_relax(r: Relaxer, n_moving: int, target: float | None = None, max_iter: int = 50,
                 krylov_tol: float = 1e-4, krylov_max: int = 3, move_cap: float = 0.25,
                 max_backtracks: int = 6, time_limit: float | None = None,
                 forcing: str | None = "ew", checkpoint_every: int = 0) -> NewtonLog:
    """Newton-MINRES on F = P a until the force residual is <= target.

    forcing = None solves every Newton system to the relative residual
    krylov_tol; forcing = "ew" picks the tolerance per step by Eisenstat and
    Walker's second rule (eta_k = 0.9 (|F_k|/|F_k-1|)^2, safeguarded, between
    krylov_tol and 0.5): loose solves far from the solution, tight ones near it.
    At most krylov_max MINRES iterations either way. checkpoint_every > 0
    keeps a device snapshot of the state every that many accepted Newton
    steps in log.checkpoint (a restart point; Relaxer.restore puts it back)."""
    h = r.h_min
    log = NewtonLog()
    t0 = time.perf_counter()
    F = projected_force(r)
    f2 = r.dot(F, F)
    log.residual.append((0.0, math.sqrt(max(f2, 0.0) / max(n_moving, 1))))
    d = torch.zeros_like(F)
    solver = _Minres(r, F)
    eta, f2_prev = 0.5, None
    for _ in range(max_iter):
        R = log.residual[-1][1]
        if target is not None and R <= target:
            break
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        log.newton_iters += 1
        if forcing == "ew":
            if f2_prev is not None:
                e = 0.9 * (f2 / f2_prev)
                safe = 0.9 * eta * eta
                eta = max(e, safe) if safe > 0.1 else e
            eta = min(0.5, max(krylov_tol, eta))
            tol = eta
        else:
            tol = krylov_tol
        f2_prev = f2
        log.krylov_iters += solver.solve(F, d, tol, krylov_max)   # A d = F, A = -PJP: d = -(PJP)^-1 F
        r.clamp(d, move_cap * h)
        snap = r.snapshot()
        s, accepted = 1.0, False
        for _bt in range(max_backtracks + 1):
            r.displace(d, s)
            r.project()
            F_new = projected_force(r)
            f2_new = r.dot(F_new, F_new)
            if math.isfinite(f2_new) and f2_new < f2:
                accepted = True
                break
            log.backtracks += 1
            r.restore(snap)
            s *= 0.5
        if not accepted:
            break
        F, f2 = F_new, f2_new
        if checkpoint_every > 0 and log.newton_iters % checkpoint_every == 0:
            log.checkpoint = r.snapshot()
        torch.cuda.synchronize()
        log.residual.append((time.perf_counter() - t0, math.sqrt(max(f2, 0.0) / max(n_moving, 1))))
    return log


def plain_relax(r: Relaxer, n_moving: int, iters: int, record_every: int = 10):
    """The plain loop of Algorithm 1 with the residual recorded every few
    iterations (its evaluation is excluded from the recorded wall time)."""
    log = []
    wall = 0.0
    b = projected_force(r)
    log.append((0.0, force_residual(r, b, n_moving)))
    done = 0
    while done < iters:
        m = min(record_every, iters - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(m):
            r.step(keep_accel=False)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        done += m
        b = projected_force(r)
        log.append((wall, force_residual(r, b, n_moving)))
    return log
