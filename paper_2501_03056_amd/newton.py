"""Newton-Krylov relaxation (trust-region Newton-CG, Steihaug) on one GPU.

The plain loop of Algorithm 1 moves every particle by dt^2 a with
dt^2 = (h/16)/max|a|: a gradient step of the pair energy E scaled so that the
fastest particle moves h/16. For one moving class with fixed other sources
the force field is a = -grad E (fppg_relax_energy), so the relaxation is an
energy minimisation that a Newton method can take in far fewer sweeps:

    b = P a                                   (tangent-space force)
    solve (P H P) d = b by CG, H v = -J v     (fppg_relax_hvp, fppg_tangent_project)
    truncated at the trust-region radius or at negative curvature (Steihaug),
    x <- Pi(x + s d)                          (fppg_displace + fppg_project)
    accept if the actual energy decrease is a fair share of the predicted one,
    adapt the radius.

H is indefinite (the pair curvature across the bond is negative), hence the
trust region. s caps the largest single-particle move at h/2 so the
projection and revert rules act on short steps as in the plain loop. Every
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
    """Rebuild the cells at the current positions and return b = P a."""
    r.build_cells()
    r.relax_step(keep_accel=True)
    b = r.accel.clone()
    r.tangent(b)
    return b


def force_residual(r: Relaxer, b: torch.Tensor, n_moving: int) -> float:
    """sqrt(mean over moving particles of |P a|^2)."""
    return math.sqrt(max(r.dot(b, b), 0.0) / max(n_moving, 1))


def _to_boundary(dd: float, dp: float, pp: float, delta: float) -> float:
    """tau >= 0 with |d + tau p| = delta."""
    a, bq, c = pp, 2.0 * dp, dd - delta * delta
    disc = max(bq * bq - 4.0 * a * c, 0.0)
    return (-bq + math.sqrt(disc)) / (2.0 * a) if a > 0 else 0.0


@dataclass
class NewtonLog:
    residual: list = field(default_factory=list)   # (wall s, R) after every accepted step
    energy: list = field(default_factory=list)
    newton_iters: int = 0
    cg_iters: int = 0
    rejected: int = 0


def newton_relax(r: Relaxer, n_moving: int, target: float | None = None, max_iter: int = 50,
                 cg_tol: float = 1e-4, cg_max: int = 60, delta0: float | None = None,
                 move_cap: float = 0.5, time_limit: float | None = None) -> NewtonLog:
    """Minimise E over the moving particles until the force residual is <= target."""
    h = r.h_min
    delta = delta0 if delta0 is not None else 0.25 * h * math.sqrt(max(n_moving, 1))
    log = NewtonLog()
    t0 = time.perf_counter()
    b = projected_force(r)
    E = r.energy()
    R = force_residual(r, b, n_moving)
    log.residual.append((0.0, R))
    log.energy.append(E)
    d = torch.zeros_like(b)
    res = torch.empty_like(b)
    p = torch.empty_like(b)
    Hp = torch.empty_like(b)
    for _ in range(max_iter):
        if target is not None and R <= target:
            break
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        log.newton_iters += 1
        # Steihaug CG on (P H P) d = b
        d.zero_()
        res.copy_(b)
        p.copy_(b)
        rz = r.dot(res, res)
        bnorm = math.sqrt(rz)
        dd = dp = 0.0
        for _k in range(cg_max):
            log.cg_iters += 1
            r.hvp(p, out=Hp)          # J p
            r.tangent(Hp)             # P J p ;  p^T H p = -p . (P J p)
            pHp = -r.dot(p, Hp)
            pp = r.dot(p, p)
            dp = r.dot(d, p)
            if pHp <= 0.0:
                r.axpby(_to_boundary(dd, dp, pp, delta), p, 1.0, d)
                break
            alpha = rz / pHp
            if dd + 2.0 * alpha * dp + alpha * alpha * pp >= delta * delta:
                r.axpby(_to_boundary(dd, dp, pp, delta), p, 1.0, d)
                break
            r.axpby(alpha, p, 1.0, d)
            r.axpby(alpha, Hp, 1.0, res)  # res <- res - alpha H p = res + alpha P J p
            dd = r.dot(d, d)
            rz_new = r.dot(res, res)
            if math.sqrt(rz_new) <= cg_tol * bnorm:
                break
            r.axpby(1.0, res, rz_new / rz, p)
            rz = rz_new
        dd = r.dot(d, d)
        # cap the largest single move, then the predicted reduction of the model
        mx = r.maxnorm(d)
        s = min(1.0, move_cap * h / mx) if mx > 0 else 0.0
        r.hvp(d, out=Hp)
        r.tangent(Hp)
        dHd = -r.dot(d, Hp)
        bd = r.dot(b, d)
        pred = s * bd - 0.5 * s * s * dHd
        snap = r.snapshot()
        r.displace(d, s)
        r.project()
        b_new = projected_force(r)
        E_new = r.energy()
        rho = (E - E_new) / pred if pred > 0 else -1.0
        if not (rho > 0.1) or not math.isfinite(E_new):
            r.restore(snap)
            delta *= 0.25
            log.rejected += 1
            if delta < 1e-6 * h:
                break
            continue
        if rho > 0.75 and math.sqrt(dd) * s >= 0.99 * delta:
            delta *= 2.0
        elif rho < 0.25:
            delta *= 0.5
        E, b = E_new, b_new
        R = force_residual(r, b, n_moving)
        torch.cuda.synchronize()
        log.residual.append((time.perf_counter() - t0, R))
        log.energy.append(E)
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
