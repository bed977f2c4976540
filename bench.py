"""Benchmark: particle-relaxation iterations per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere|cube|gear]

A step is one iteration of the relaxation loop (Algorithm 1 of arXiv
2501.03056): cell rebuild, forces + time step + displacement, projection.
Default workload: icosphere of radius 1 (subdivision level 5, 20,480 facets),
dx = 0.01, h = 1.3 dx: ~4.13 M volume + 125,664 surface particles, all moving,
synthetic and seeded (the paper's models are not available).

Prints ONE JSON line with the whole-job throughput (particle-updates/s), the
pair-evaluation rate, the force kernel's roofline figures (timed with HIP
events on its launch stream, inside the timed region) and the CPU oracle timed
on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X vector FP32 (published)
PEAK_HBM_GBS = 8000.0
FLOPS_PER_PAIR = 19               # see roofline_note()
KERNEL_SOURCES = ["paper_2501_03056_amd/csrc/force.hip", "paper_2501_03056_amd/csrc/internal.h",
                  "paper_2501_03056_amd/csrc/stencil.h"]


def roofline_note():
    return ("algorithmic work of the force kernel = true (receiver, source) pairs x 19 flops: "
            "3 sub + 3 mul + 2 add (squared distance), 1 sqrt, 1 fma (1 - r/2h), 2 mul (cube), "
            "3 fma (accumulate); candidates rejected by the predicate are not counted")


# Algorithmic HBM bytes of the streaming phases (each particle or cell read or
# written once, as the kernels are designed to do): cell rebuild 112 B per
# particle (pos 16 read; key + rank 8 written, 8 read; scatter 20; final
# gather 48 + 12) + 12 B per cell (count, scan, cell_start); update 52 B per
# launched particle (pos, accel, owner read, disp written); projection 48 B per
# moving particle (pos and disp read, pos written) + 8 B per surface particle
# (owner read and written); force 32 B per moving receiver (own pos read,
# accel written; the sources are re-read from cache).
BUILD_B_PER_PARTICLE, BUILD_B_PER_CELL = 112, 12
UPDATE_B, PROJECT_B, PROJECT_SURF_B, FORCE_B = 52, 48, 8, 32


def valu_issue(kernel_hash, force_ms, pairs):
    """VALU lane-operations per second of the force kernel: the counted VALU
    instructions per launch (SQ_INSTS_VALU of the committed counter summary) x
    64 lanes / the live launch time, against the non-packed issue peak."""
    insts = profile_value(kernel_hash, "valu_insts_per_launch")
    if insts is None:
        return None
    rate = insts * 64 / (force_ms / 1e3)
    return {"valu_insts_per_launch": insts, "lane_ops_per_s": rate, "single_issue_peak": VALU_LANE_OPS_PEAK,
            "frac": rate / VALU_LANE_OPS_PEAK, "lane_slots_per_true_pair": insts * 64 / pairs,
            "note": "instruction issue (dual issue lets it pass 1), not algorithmic flops"}


def hbm_phases(wl, ncell, n_moving, phase_ms, ms_step):
    """Achieved GB/s of algorithmic bytes per phase against the 8 TB/s HBM
    peak (phase times from the event-timed breakdown pass), and for the whole
    step with the force kernel's own bytes included."""
    n_surf = int(np.sum(np.asarray(wl.tag) == 2))
    bytes_ = {"build_cells": BUILD_B_PER_PARTICLE * wl.n + BUILD_B_PER_CELL * ncell,
              "update": UPDATE_B * wl.n,
              "project": PROJECT_B * n_moving + PROJECT_SURF_B * n_surf,
              "force": FORCE_B * n_moving}
    out = {}
    for k, b in bytes_.items():
        if k in phase_ms and phase_ms[k] > 0:
            gbs = b / (phase_ms[k] / 1e3) / 1e9
            out[k] = {"bytes": b, "ms": phase_ms[k], "GB/s": gbs, "frac": gbs / PEAK_HBM_GBS}
    step_b = sum(bytes_.values())
    gbs = step_b / (ms_step / 1e3) / 1e9
    out["step"] = {"bytes": step_b, "ms": ms_step, "GB/s": gbs, "frac": gbs / PEAK_HBM_GBS,
                   "note": "the step is bound by the force kernel's instruction issue, not by HBM"}
    return out


def make_workload(name, k=2, slab=0):
    import synth
    if name == "sphere":
        wl, wname = synth.sphere_workload(level=5, dx=0.01, seed=2, k=k), "icosphere_l5_r1_dx0.01_h1.3dx"
    elif name == "cube":
        wl, wname = synth.cube_workload(n=24, seed=1, k=k), "unit_cube_dx1/24_h1.3dx"
    else:
        raise SystemExit(f"unknown workload {name}")
    for g in wl.geoms:
        g.slab = slab
    return wl, wname


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def profile_value(kernel_hash, key):
    """A per-launch figure of the force kernel measured by rocprofv3 counters
    (the committed summary's `kernel_source_hash:` line and the `key:` line),
    or None if absent or taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "force_sphere_l5_counters.md")
    if not os.path.exists(p):
        return None
    text = open(p).read()
    h = re.search(r"^kernel_source_hash:\s*(\S+)", text, re.M)
    b = re.search(r"^" + key + r":\s*(\d+)", text, re.M)
    if not h or not b or h.group(1) != kernel_hash:
        return None
    return int(b.group(1))


def traffic_from_profile(kernel_hash):
    """HBM bytes per force launch (FETCH_SIZE and WRITE_SIZE, calibrated)."""
    return profile_value(kernel_hash, "hbm_bytes_per_launch")


# Non-packed VALU issue: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
# (the build keeps packed FP32 off); dual issue can exceed it.
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9


def cpu_baseline(wl, sample=160, seed=0):
    """The oracle (brute force, FP64) on a bounded sample of the same step:
    forces of `sample` moving receivers against all particles, then their
    projection / inside test. Reported rate = sampled particle-updates / s."""
    from oracle import force as oforce
    from oracle import geometry as ogeo
    from oracle import step as ostep
    from threadpoolctl import threadpool_limits
    rng = np.random.Generator(np.random.PCG64(seed))
    mov = np.nonzero(oforce.moving_mask(wl.tag, wl.move_mask))[0]
    rec = np.sort(rng.choice(mov, size=min(sample, len(mov)), replace=False))
    with threadpool_limits(limits=1):          # one core: numpy and any BLAS it calls
        t0 = time.perf_counter()
        a, S, cnt = oforce.accel(wl, rec)
        # the step needs amax over all particles; the sample uses its own max (same cost per particle)
        tau = (float(wl.geoms[0].h) / 16.0) / max(np.linalg.norm(a, axis=1).max(), 1e-300)
        y = wl.pos[rec].astype(np.float64) + tau * a
        s = wl.tag[rec] == 2
        if s.any():
            ostep.project_surface(wl, y[s], 0)
        v = wl.tag[rec] == 3
        if v.any():
            ogeo.winding_number(y[v], wl.geoms[0].mesh.vert, wl.geoms[0].mesh.tri)
        dt = time.perf_counter() - t0
    return {"value": len(rec) / dt, "unit": "particle-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(rec)} random moving particles of the same workload: brute-force forces against "
                      f"all {wl.n} particles, FP64 projection over all facets or winding-number inside test "
                      f"({dt:.1f} s, numpy single thread)"}


def bench_generate(args):
    """The generation front end (fppg_generate: background-grid classes and the
    initial particles) on the 24-tooth gear mesh at spacing --gear-dx; value =
    background cells classified per second (the call's wall time, device
    temporaries and host-device copies included; best of 3)."""
    import torch
    from synth import meshes as M
    from paper_2501_03056_amd import Context
    from paper_2501_03056_amd.front import generate
    dx = args.gear_dx
    mesh = M.gear()
    lo, hi = mesh.vert.min(0) - 2 * dx, mesh.vert.max(0) + 2 * dx
    dims = tuple(int(v) for v in np.ceil((hi - lo) / dx))
    ctx = Context(0)
    cap = int(np.prod(dims))
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cls, pos, owner = generate(mesh.vert, mesh.tri, dx, lo, dims, ctx=ctx, cap=cap)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    tags = (pos[:, 3].contiguous().view(torch.int32) & 7).cpu().numpy()
    ncell = int(np.prod(dims))
    t = min(times)
    out = {"metric": "background cells classified/s", "value": ncell / t, "unit": "cells/s", "n_gpus": 1,
           "steps": 3, "warmup": 0, "ms_per_step": 1e3 * t, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"gear24_generate_dx{dx:g}", "facets": int(len(mesh.tri)), "dims": list(dims),
                      "cells": ncell},
           "particles": {"volume": int(np.sum(tags == 3)), "surface": int(np.sum(tags == 2))},
           "cell_classes": {k: int(v) for k, v in zip(("external", "internal", "surface"),
                                                       np.bincount(cls.cpu().numpy().ravel(), minlength=3))},
           "seconds_all": times}
    print(json.dumps(out), flush=True)


def bench_features(args):
    """Feature extraction (fppg_features: feature edges, singular vertices,
    lines and loops, feature-line particles at spacing --gear-dx) on the
    24-tooth gear mesh; value = facets processed per second (the call's wall
    time with its size query, device temporaries and copies; best of 3)."""
    import math
    import torch
    from synth import meshes as M
    from paper_2501_03056_amd import Context
    from paper_2501_03056_amd.front import features
    dx = args.gear_dx
    mesh = M.gear()
    ctx = Context(0)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = features(mesh.vert, mesh.tri, math.cos(math.radians(30.0)), dx, ctx=ctx)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = min(times)
    out = {"metric": "facets processed/s (feature extraction)", "value": len(mesh.tri) / t, "unit": "facets/s",
           "n_gpus": 1, "steps": 3, "warmup": 0, "ms_per_step": 1e3 * t, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"gear24_features_dx{dx:g}", "facets": int(len(mesh.tri)), "threshold_deg": 30.0},
           "features": {"edges": int(len(f["edges"])), "singular": int(len(f["singular"])),
                        "lines": int(len(f["line_closed"])), "particles": int(len(f["pos"]))},
           "seconds_all": times}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """64 independent solids (boxes and cylinders, 5k-500k particles each) in
    one launch per kernel; stencil half-width, launch mode (eager or HIP
    graph replay) and the force kernel's launch shape autotuned; value = the
    chosen configuration, the other mode reported beside it."""
    import torch
    import synth
    from paper_2501_03056_amd import Relaxer
    from paper_2501_03056_amd.tune import autotune, regrid
    t0 = time.perf_counter()
    wl = synth.workload.batch_workload(n_geom=64, seed=4000)
    print(f"[bench] batch: {wl.n} particles in {len(wl.geoms)} geometries, built in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    tune = autotune(wl, cache=os.path.join(os.environ.get("TMPDIR", "/tmp"), "fppg_autotune.json"))
    print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    r = Relaxer(regrid(wl, tune["k"]), device=0)
    r.ctx.set_launch(tune["force_block"], tune["xcd_remap"])
    for _ in range(args.warmup):
        r.step(keep_accel=False)
    r.profile(True)
    for _ in range(10):
        r.step(keep_accel=False)
    prof = r.profile_read()
    r.profile(False)
    steps = args.steps - (args.steps % 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        r.step(keep_accel=False)
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    r.capture(iters=2)
    r.replay(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.replay(steps // 2)
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t0) / steps
    r.release_graph()
    ms = graph_ms if tune["mode"] == "graph" else eager_ms
    n_moving = wl.n_moving()
    out = {"metric": "particle-updates/s per relaxation step", "value": n_moving / (ms / 1e3),
           "unit": "particle-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch64_boxes_cylinders_seed4000", "geometries": len(wl.geoms),
                      "particles": wl.n, "moving": n_moving, "autotune": tune},
           "kernels_ms_per_step_eager": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]},
           "eager_ms_per_step": eager_ms, "graph_ms_per_step": graph_ms,
           "device_status": r.read_status()}
    print(json.dumps(out), flush=True)


def bench_gear(args):
    """The gear relaxed in three tiers (feature lines, then surface, then
    volume particles; the other classes are fixed sources of the moving one),
    --tier-iters iterations each on the same state. value = sum over tiers of
    moving particles x iterations / total seconds. Then the three-layer
    variant of the volume tier (section 3.3.4): the volume particles deeper
    than --layer-width dx become a fixed core and only the layer above it
    relaxes (reported under "three_layer", with the feature and surface tiers,
    and not in value)."""
    import torch
    import synth
    from paper_2501_03056_amd import Relaxer
    dx = args.gear_dx
    t0 = time.perf_counter()
    gen = None
    if args.gear_source == "pipeline":
        # the particles from the GPU front end (feature extraction + generation)
        from synth import meshes as M
        from paper_2501_03056_amd import Context, pipeline
        ctx = Context(0)
        mesh = M.gear()
        pipeline.from_mesh(mesh.vert, mesh.tri, dx, ctx=ctx)          # warm-up (kernel loading)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wl = pipeline.from_mesh(mesh.vert, mesh.tri, dx, ctx=ctx)
        torch.cuda.synchronize()
        gen = {"seconds": time.perf_counter() - t0, "note": "fppg_features + fppg_generate + host assembly"}
    else:
        wl = synth.gear_workload(dx=dx, seed=3, k=args.k)
    for g in wl.geoms:
        g.slab = args.slab
    print(f"[bench] gear dx={dx:g}: {wl.n} particles {wl.counts()} built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    r = Relaxer(wl, device=0)
    print(f"[bench] geometry on the device in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    tiers = [("feature", 1 << synth.FEATURE), ("surface", 1 << synth.SURFACE), ("volume", 1 << synth.VOLUME),
             ("volume_layer", 1 << synth.VOLUME)]
    out_tiers, total_s, total_upd = {}, 0.0, 0.0
    layer = {}
    for name, mm in tiers:
        if name == "volume_layer":
            # three-layer volume relaxation (section 3.3.4): the volume particles
            # deeper than the layer width become the fixed core
            width = args.layer_width * dx
            layer = {"width": width, "width_dx": args.layer_width, "core": r.volume_layers(width)}
            print(f"[bench] volume layer: width {width:g}, {layer['core']} particles fixed as the core",
                  file=sys.stderr, flush=True)
        # a sparse tier leaves out the particles it does not reach (rank above
        # its moving class: neither receivers nor sources)
        r.tier(mm, compact=not args.no_compact)
        n_moving = r.n_moving()
        # a sparse tier launches only its moving particles' lanes
        r.use_list = not args.no_list and n_moving < r.na // 2
        for _ in range(args.warmup):
            r.step(keep_accel=False)
        r.build_cells()
        r.accel.zero_()   # a receiver list leaves the other rows unwritten
        r.relax_step(count_pairs=True)
        pairs = float(r.accel[:, 3].double().sum().item())
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.tier_iters):
            r.step(keep_accel=False)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        r.profile(True)   # per-phase breakdown from a separate pass
        for _ in range(min(args.tier_iters, 20)):
            r.step(keep_accel=False)
        prof = r.profile_read()
        r.profile(False)
        if name != "volume_layer":
            total_s += ms / 1e3
            total_upd += n_moving * args.tier_iters
        out_tiers[name] = {"moving": n_moving, "iters": args.tier_iters, "ms_per_step": ms / args.tier_iters,
                           "particle_updates_per_s": n_moving * args.tier_iters / (ms / 1e3),
                           "pairs_per_step": pairs, "pair_evals_per_s": pairs * args.tier_iters / (ms / 1e3),
                           "receiver_list": bool(r.use_list), "active_particles": r.na,
                           "kernels_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}}
        print(f"[bench] tier {name}: {n_moving} moving of {r.na} active, {ms / args.tier_iters:.3f} ms/step",
              file=sys.stderr,
              flush=True)
    t3 = [out_tiers[k] for k in ("feature", "surface", "volume_layer")]
    three_layer = {"particle_updates_per_s": sum(t["moving"] * t["iters"] for t in t3)
                   / sum(t["ms_per_step"] * t["iters"] / 1e3 for t in t3), **layer}
    out = {"metric": "particle-updates/s", "value": total_upd / total_s, "unit": "particle-updates/s",
           "n_gpus": 1, "steps": 3 * args.tier_iters, "warmup": 3 * args.warmup,
           "ms_per_step": 1e3 * total_s / (3 * args.tier_iters), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"gear24_dx{dx:g}_tiers_feature_surface_volume"
                                  + ("_gpu_generated" if gen else ""), "particles": wl.n, "generation": gen,
                      "counts": wl.counts(), "facets": int(r.geom.n_tri), "stencil_k": int(wl.geoms[0].k),
                      "key_slab_rows": int(args.slab)},
           "tiers": out_tiers, "three_layer": three_layer, "device_status": r.read_status()}
    print(json.dumps(out), flush=True)


def _first_at_or_below(curve, target):
    for t, R in curve:
        if R <= target:
            return t
    return None


def bench_newton(args):
    """Newton-Krylov vs the plain loop on one tier (--newton-tier: by default
    the volume tier, where volume particles move and surface, feature and
    singular particles are fixed sources; on the gear also the surface or the
    feature tier, each after the tier partition), from the
    same initial state: the plain loop runs --plain-iters iterations (the
    paper's fixed iteration count) and its final force residual R_plain is the
    target; Newton-MINRES runs until R <= R_plain. value = plain seconds /
    Newton seconds. The plain loop's residual is not monotone (its step keeps
    the fastest particle moving h/16), so the first time it dips to R_plain
    and its best residual are reported as well."""
    import torch
    import synth
    from paper_2501_03056_amd import Relaxer
    from paper_2501_03056_amd.newton import newton_relax, plain_relax
    tier = args.newton_tier
    mm = 1 << {"volume": synth.VOLUME, "surface": synth.SURFACE, "feature": synth.FEATURE}[tier]
    if tier != "volume" and args.newton_workload != "gear":
        raise SystemExit("--newton-tier surface/feature needs the gear (the sphere has no feature lines)")
    if args.newton_workload == "gear":
        dx = args.newton_dx or 0.004
        wl, wname = synth.gear_workload(dx=dx, seed=3, k=args.k, move_mask=mm), f"gear24_dx{dx:g}_{tier}_tier"
    else:
        dx = args.newton_dx or 0.01
        wl, wname = synth.sphere_workload(level=5, dx=dx, seed=2, k=args.k, move_mask=mm), \
            f"icosphere_l5_dx{dx:g}_volume_tier"
    n_moving = wl.n_moving()
    print(f"[bench] newton {wname}: {wl.n} particles, {n_moving} moving", file=sys.stderr, flush=True)
    rp = Relaxer(wl, device=0)
    rp.tier(mm)   # a feature or surface tier leaves out the particles it does not reach
    plain = plain_relax(rp, n_moving, iters=args.plain_iters, record_every=1)
    target, t_plain = plain[-1][1], plain[-1][0]
    t_first = _first_at_or_below(plain, target)
    best = min(range(len(plain)), key=lambda q: plain[q][1])
    print(f"[bench] plain: R {plain[0][1]:.4g} -> {target:.4g} after {args.plain_iters} iterations "
          f"({t_plain:.4f}s; first at or below it {t_first:.4f}s); best {plain[best][1]:.4g} at iteration {best}",
          file=sys.stderr, flush=True)
    del rp
    rn = Relaxer(wl, device=0)
    rn.tier(mm)
    torch.cuda.synchronize()
    kw = dict(forcing="ew", krylov_tol=1e-4, krylov_max=args.krylov_max, checkpoint_every=10)
    log = newton_relax(rn, n_moving, target=target, max_iter=500, time_limit=20 * t_plain + 20, **kw)
    t_newton = log.residual[-1][0]
    reached = log.residual[-1][1] <= target
    print(f"[bench] newton: R {log.residual[-1][1]:.4g} at {t_newton:.4f}s ({log.newton_iters} Newton, "
          f"{log.krylov_iters} MINRES iterations)", file=sys.stderr, flush=True)
    # continue from there to the plain loop's best residual, then for the plain loop's whole time
    more = newton_relax(rn, n_moving, target=plain[best][1], max_iter=500, time_limit=20 * t_plain + 20, **kw)
    t_best = t_newton + more.residual[-1][0] if more.residual[-1][1] <= plain[best][1] else None
    rest = newton_relax(rn, n_moving, target=None, max_iter=500,
                        time_limit=max(t_plain - (t_best or t_newton), 0.0), **kw)
    out = {"metric": "Newton-HVP vs plain s to residual", "value": t_plain / t_newton if reached else 0.0,
           "unit": "x (plain-loop seconds for its iterations / Newton seconds to the same force residual)",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wname, "particles": wl.n, "moving": n_moving,
                      "plain_iters": args.plain_iters, "krylov": "MINRES", "forcing": "Eisenstat-Walker 2",
                      "krylov_tol_min": 1e-4, "krylov_max": args.krylov_max, "move_cap": "h/4",
                      "newton_checkpoint_every": 10},
           "plain": {"seconds": t_plain, "R0": plain[0][1], "R_final": target,
                     "seconds_first_at_or_below_R_final": t_first,
                     "R_best": plain[best][1], "iters_to_best": best, "seconds_to_best": plain[best][0],
                     "curve": plain[::max(1, len(plain) // 50)]},
           "newton": {"seconds": t_newton, "R": log.residual[-1][1], "reached": reached,
                      "newton_iters": log.newton_iters, "krylov_iters": log.krylov_iters,
                      "backtracks": log.backtracks, "curve": log.residual,
                      "seconds_to_plain_best": t_best,
                      "R_after_plain_seconds": rest.residual[-1][1]},
           "ratios": {"vs_plain_first_arrival": (t_first / t_newton) if reached and t_first else None,
                      "vs_plain_best": (plain[best][0] / t_best) if t_best else None},
           "device_status": rn.read_status()}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="step", choices=["step", "batch", "newton", "gear", "generate", "features"])
    ap.add_argument("--gear-dx", type=float, default=0.004)
    ap.add_argument("--tier-iters", type=int, default=100)
    ap.add_argument("--gear-source", default="synth", choices=["synth", "pipeline"],
                    help="gear: particles from the synthetic generator or from the GPU front end")
    ap.add_argument("--layer-width", type=float, default=3.0,
                    help="gear: width of the relaxed volume layer in units of dx (three-layer tier)")
    ap.add_argument("--no-list", action="store_true",
                    help="gear tiers: launch every particle's lane instead of the moving-particle list")
    ap.add_argument("--no-compact", action="store_true",
                    help="gear tiers: keep every particle active (no tier partition)")
    ap.add_argument("--plain-iters", type=int, default=100)
    ap.add_argument("--newton-dx", type=float, default=None, help="default 0.004 (gear), 0.01 (sphere)")
    ap.add_argument("--newton-workload", default="gear", choices=["gear", "sphere"])
    ap.add_argument("--krylov-max", type=int, default=3)
    ap.add_argument("--newton-tier", default="volume", choices=["volume", "surface", "feature"])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sphere")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=960)
    ap.add_argument("--k", type=int, default=2, help="stencil half-width of the particle cells (1 or 2)")
    ap.add_argument("--slab", type=int, default=0,
                    help="cell rows per slab of the cell key (0: one slab per geometry)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device to device first (reference kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding over GPUs "
              "(geometries, or key slabs with a halo exchange) is not built", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "generate":
        return bench_generate(args)
    if args.mode == "features":
        return bench_features(args)
    if args.mode == "newton":
        return bench_newton(args)
    if args.mode == "gear":
        return bench_gear(args)
    import torch
    from paper_2501_03056_amd import Relaxer

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    wl, wname = make_workload(args.workload, args.k, args.slab)
    print(f"[bench] workload {wname}: {wl.n} particles {wl.counts()} built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    r = Relaxer(wl, device=0)
    n_moving = wl.n_moving()
    for _ in range(args.warmup):
        r.step(keep_accel=False)
    # true pair count (separate counting pass, not timed)
    r.build_cells()
    r.relax_step(count_pairs=True)
    r.project()
    pairs0 = float(r.accel[:, 3].double().sum().item())
    torch.cuda.synchronize()
    print(f"[bench] warmup done, {pairs0:.4g} pairs/step", file=sys.stderr, flush=True)

    # timed region: HIP events on the launch stream bracket the force kernel
    # only (the roofline's kernel); the per-phase breakdown comes from a
    # separate pass, since every event pair adds a little time to the stream
    r.profile(True, phases=("force",))
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        r.step(keep_accel=False)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = start.elapsed_time(stop)
    force_prof = r.profile_read()["force"]
    r.profile(True)
    for _ in range(min(args.steps, 50)):
        r.step(keep_accel=False)
    prof = r.profile_read()
    r.profile(False)
    r.build_cells()
    r.relax_step(count_pairs=True)
    pairs1 = float(r.accel[:, 3].double().sum().item())
    status = r.read_status()
    pairs = 0.5 * (pairs0 + pairs1)

    ms_step = ms / args.steps
    value = n_moving * args.steps / (ms / 1e3)
    f_ms, f_n = force_prof
    force_ms = f_ms / max(f_n, 1)
    achieved = pairs * FLOPS_PER_PAIR / (force_ms / 1e3) / 1e12
    khash = source_hash(KERNEL_SOURCES)
    traffic = traffic_from_profile(khash)
    phase_ms = {k: (v[0] / max(v[1], 1)) for k, v in prof.items() if v[1]}
    hbm = hbm_phases(wl, int(r.geom.ncell), n_moving, phase_ms, ms_step)
    out = {
        "metric": "particle-updates/s per relaxation step",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "particles": wl.n, "moving": n_moving, "facets": int(r.geom.n_tri),
                   "stencil_k": int(wl.geoms[0].k), "key_slab_rows": int(args.slab), "h_over_dx": 1.3,
                   "pairs_per_step": pairs},
        "pair_evals_per_s": pairs * args.steps / (ms / 1e3),
        "kernels_ms_per_step": phase_ms,
        "hbm_phases": hbm,
        "roofline": {"bound": "alu", "kernel": "k_force", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "work_per_launch": pairs * FLOPS_PER_PAIR, "avg_launch_ms": force_ms,
                     "kernel_source_hash": khash, "valu_issue": valu_issue(khash, force_ms, pairs)},
        "device_status": status,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
