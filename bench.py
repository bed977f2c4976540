"""Benchmark: particle-relaxation iterations per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one iteration of the relaxation loop (Algorithm 1 of arXiv
2501.03056): cell rebuild, forces + time step + displacement, projection.
Default workload: the 24-tooth gear on its full mesh (207,360 facets), dx =
0.004, h = 1.3 dx, 12.4 M particles (11.8 M volume, 0.54 M surface, 13 k
feature, 192 singular), synthetic and seeded (the paper's models are not
available); the timed steps are its volume tier (volume particles move, the
other classes are fixed sources), the largest single-GPU configuration and the
one whose state exceeds the MI355X's 256 MB Infinity Cache.

Prints ONE JSON line with the whole-job throughput (particle-updates/s), the
pair-evaluation rate, the force kernel's roofline figures (timed with HIP
events on its launch stream, inside the timed region), the feature and surface
tiers of the same gear, the Newton-Krylov form against the plain loop on the
volume tier (seconds to the plain loop's residual, against its first arrival
there), the icosphere workload as a secondary line, and the CPU oracle timed
on a bounded sample of the same workload on all host cores.
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


def valu_issue(kernel_hash, force_ms, pairs, profile=None):
    """VALU lane-operations per second of the force kernel: the counted VALU
    instructions per launch (SQ_INSTS_VALU of the committed counter summary) x
    64 lanes / the live launch time, against the non-packed issue peak."""
    insts = profile_value(kernel_hash, "valu_insts_per_launch", profile)
    if insts is None:
        return None
    rate = insts * 64 / (force_ms / 1e3)
    return {"valu_insts_per_launch": insts, "lane_ops_per_s": rate, "single_issue_peak": VALU_LANE_OPS_PEAK,
            "frac": rate / VALU_LANE_OPS_PEAK, "lane_slots_per_true_pair": insts * 64 / pairs,
            "note": "instruction issue (dual issue lets it pass 1), not algorithmic flops"}


def hbm_phases(n_active, ncell, n_moving, n_surf_moving, phase_ms, ms_step):
    """Achieved GB/s of algorithmic bytes per phase against the 8 TB/s HBM
    peak (phase times from the event-timed breakdown pass), and for the whole
    step with the force kernel's own bytes included."""
    bytes_ = {"build_cells": BUILD_B_PER_PARTICLE * n_active + BUILD_B_PER_CELL * ncell,
              "update": UPDATE_B * n_active,
              "project": PROJECT_B * n_moving + PROJECT_SURF_B * n_surf_moving,
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


COUNTER_PROFILE = "force_gear_volume_counters.md"


def profile_value(kernel_hash, key, profile=None, launch=None):
    """A per-launch figure of the force kernel measured by rocprofv3 counters
    (the committed summary's `kernel_source_hash:` line and the `key:` line),
    or None if absent, taken on a different kernel source, or (launch given as
    "block,remap,persistent") taken in a different launch shape (the summary's
    `force_launch:` line)."""
    p = os.path.join(ROOT, "profiles", profile or COUNTER_PROFILE)
    if not os.path.exists(p):
        return None
    text = open(p).read()
    h = re.search(r"^kernel_source_hash:\s*(\S+)", text, re.M)
    b = re.search(r"^" + key + r":\s*(\d+)", text, re.M)
    if not h or not b or h.group(1) != kernel_hash:
        return None
    if launch is not None:
        lm = re.search(r"^force_launch:\s*(\S+)", text, re.M)
        if not lm or lm.group(1) != launch:
            return None
    return int(b.group(1))


def traffic_from_profile(kernel_hash, profile=None, launch=None):
    """HBM bytes per force launch (FETCH_SIZE and WRITE_SIZE, calibrated)."""
    return profile_value(kernel_hash, "hbm_bytes_per_launch", profile, launch)


# Non-packed VALU issue: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
# (the build keeps packed FP32 off); dual issue can exceed it.
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9


def host_cores():
    """CPUs this process may run on (at most 16, the host share of one GPU)
    and the CPU model name."""
    n = min(16, len(os.sched_getaffinity(0)))
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


def cpu_baseline(wl, sample=1 << 20, seed=0):
    """The oracle's full-size mode (oracle/local.py: FP64 forces over candidate
    neighbour cells, the projection over candidate facets, the volume rule by
    the ray winding number) on a bounded sample of the same step: forces of
    `sample` random moving particles against all particles, then their
    displacement and projection or volume rule, on all host cores (threads).
    Reported rate = sampled particle-updates / s."""
    from oracle import force as oforce
    from oracle import local as olocal
    cores, model = host_cores()
    rng = np.random.Generator(np.random.PCG64(seed))
    mov = np.nonzero(oforce.moving_mask(wl.tag, wl.move_mask))[0]
    rec = np.sort(rng.choice(mov, size=min(sample, len(mov)), replace=False))
    t0 = time.perf_counter()
    a, S, cnt = olocal.accel(wl, receivers=rec, threads=cores)
    # the step needs amax over all movers; the sample uses its own (same cost per particle)
    tau = (float(wl.geoms[0].h) / 16.0) / max(np.linalg.norm(a, axis=1).max(), 1e-300)
    y = wl.pos[rec].astype(np.float64) + tau * a
    s = wl.tag[rec] == 2
    if s.any():
        olocal.project_surface(wl, y[s], 0)
    v = wl.tag[rec] == 3
    if v.any():
        olocal.volume_rule(y[v], wl.geoms[0].mesh)
    dt = time.perf_counter() - t0
    return {"value": len(rec) / dt, "unit": "particle-updates/s", "cores": cores, "cpu_model": model,
            "kind": "oracle",
            "sample": f"{len(rec)} random moving particles of the same workload: FP64 forces over the candidate "
                      f"neighbour cells of all {wl.n} particles, then their projection or volume rule "
                      f"({dt:.1f} s on {cores} threads; the oracle's full-size mode, pinned to its brute force)"}


def bench_generate(args):
    """The generation front end (fppg_generate: background-grid classes and the
    initial particles) on the 24-tooth gear mesh at spacing --gear-dx; value =
    background cells classified per second (the call's wall time, device
    temporaries and host-device copies included; best of 3). The same
    particles through the sparse storage (fppg_generate_sparse) are timed
    beside it and compared bit for bit."""
    import torch
    from synth import meshes as M
    from paper_2501_03056_amd import Context
    from paper_2501_03056_amd.front import generate, generate_sparse
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
    # the same particles through the sparse cell storage (no per-cell class array)
    sparse_times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        spos, sowner, sinfo = generate_sparse(mesh.vert, mesh.tri, dx, lo, dims, ctx=ctx, cap=len(pos))
        torch.cuda.synchronize()
        sparse_times.append(time.perf_counter() - t0)
    same = bool(torch.equal(spos.view(torch.int32), pos.view(torch.int32)) and torch.equal(sowner, owner))
    del spos, sowner
    out = {"metric": "background cells classified/s", "value": ncell / t, "unit": "cells/s", "n_gpus": 1,
           "steps": 3, "warmup": 0, "ms_per_step": 1e3 * t, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"gear24_generate_dx{dx:g}", "facets": int(len(mesh.tri)), "dims": list(dims),
                      "cells": ncell},
           "particles": {"volume": int(np.sum(tags == 3)), "surface": int(np.sum(tags == 2))},
           "cell_classes": {k: int(v) for k, v in zip(("external", "internal", "surface"),
                                                       np.bincount(cls.cpu().numpy().ravel(), minlength=3))},
           "seconds_all": times,
           "sparse": {"ms": 1e3 * min(sparse_times), "cells_per_s": ncell / min(sparse_times),
                      "equal_to_dense": same, "seconds_all": sparse_times, **sinfo}}
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


def graph_vs_eager(wl, steps):
    """ms per iteration of eager launches and of HIP-graph replay on one workload."""
    import torch
    from paper_2501_03056_amd import Relaxer
    r = Relaxer(wl, device=0)
    for _ in range(10):
        r.step(keep_accel=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.step(keep_accel=False)
    torch.cuda.synchronize()
    eager = 1e3 * (time.perf_counter() - t0) / steps
    r.capture(iters=2)
    r.replay(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.replay(steps // 2)
    torch.cuda.synchronize()
    graph = 1e3 * (time.perf_counter() - t0) / (2 * (steps // 2))
    r.release_graph()
    return {"eager_ms_per_step": eager, "graph_ms_per_step": graph, "particles": wl.n}


def bench_batch(args):
    """64 independent Boolean assemblies (unions and differences of 2-6 random
    boxes and cylinders, 5k-500k particles each, section 3.2.3) in one launch
    per kernel; stencil half-width, launch mode (eager or HIP graph replay),
    the force kernel's launch shape and its schedule (one block per chunk or
    persistent blocks taking tickets) autotuned; value = the chosen
    configuration, the others reported beside it. Also the cube of dx = 1/24
    eager and replayed, where launch latency and not kernel time sets the
    iteration."""
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
    r.ctx.set_launch(tune["force_block"], tune["xcd_remap"], tune["persistent"])
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
    import synth as _s
    small = graph_vs_eager(_s.cube_workload(n=24, seed=1), 400)
    out = {"metric": "particle-updates/s per relaxation step", "value": n_moving / (ms / 1e3),
           "unit": "particle-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "small_geometry_cube_dx1_24": small,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch64_boolean_assemblies_seed4000", "geometries": len(wl.geoms),
                      "assemblies": {op: sum(a["op"] == op for a in wl.meta["assemblies"])
                                     for op in ("union", "difference")},
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


def krylov_cap(asked, tier):
    """MINRES iterations per Newton step: as asked, or the tier's default (a
    volume tier gains most from cheap steps: 1.13x the plain loop's first
    arrival on the gear with 1, 0.94x with 2, 0.81x with 3; a surface tier
    from fuller solves: 0.89x with 1, 2.7x with 2, 4.1x with 3)."""
    return asked if asked > 0 else (1 if tier == "volume" else 3)


def _first_at_or_below(curve, target):
    for t, R in curve:
        if R <= target:
            return t
    return None


def bench_multires(args):
    """Two-level icosphere (level-5 mesh, coarse dx = 0.02 inside, a fine shell
    of spacing 0.01 and the surface at 0.01: multi-resolution levels 0 and 1)
    against the single-resolution sphere at the fine spacing everywhere (the
    secondary workload of the default line): the same surface resolution with
    fewer particles. value = the two-level run's particle-updates/s."""
    import torch
    import synth
    from paper_2501_03056_amd import Relaxer
    t0 = time.perf_counter()
    wl = synth.workload.multires_sphere_workload(level=5, dx=0.02, shell=2.0)
    print(f"[bench] two-level sphere: {wl.n} particles (levels {np.bincount(wl.level).tolist()}) built in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    r = Relaxer(wl, device=0)
    t = timed_steps(r, args.steps, args.warmup, "two-level sphere")
    n_mov = r.n_moving()
    del r
    wf, _ = make_workload("sphere", k=args.k)
    rf = Relaxer(wf, device=0)
    tf = timed_steps(rf, args.steps, args.warmup, "sphere at the fine spacing")
    nf = rf.n_moving()
    out = {"metric": "particle-updates/s per relaxation step", "value": n_mov * args.steps / (t["ms"] / 1e3),
           "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t["ms_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "icosphere_l5_two_levels_dx0.02_shell0.01", "particles": wl.n, "moving": n_mov,
                      "levels": np.bincount(wl.level).tolist(), "pairs_per_step": t["pairs"]},
           "force_kernel_ms": t["force_ms"], "kernels_ms_per_step": t["phase_ms"],
           "fine_everywhere": {"workload": "icosphere_l5_r1_dx0.01", "particles": wf.n, "ms_per_step": tf["ms_step"],
                               "force_kernel_ms": tf["force_ms"], "pairs_per_step": tf["pairs"],
                               "particle_updates_per_s": nf * args.steps / (tf["ms"] / 1e3)},
           "device_status": t["status"]}
    print(json.dumps(out), flush=True)


def bench_newton(args):
    """Newton-Krylov vs the plain loop on one tier (--newton-tier: by default
    the volume tier, where volume particles move and surface, feature and
    singular particles are fixed sources; on the gear also the surface or the
    feature tier, each after the tier partition), from the
    same initial state: the plain loop runs --plain-iters iterations (the
    paper's fixed iteration count) and its final force residual R_plain is the
    target; Newton-MINRES runs until R <= R_plain. The plain loop's residual
    is not monotone (its step keeps the fastest particle moving h/16): value =
    the seconds at which it FIRST dips to R_plain / Newton's seconds to it; the
    ratio to its full run and to its best residual are reported as well."""
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
    kw = dict(forcing="ew", krylov_tol=1e-4, krylov_max=krylov_cap(args.krylov_max, tier), checkpoint_every=10)
    _warm_newton(rn, n_moving, kw)
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
    out = {"metric": "Newton-HVP vs plain s to residual",
           "value": (t_first / t_newton) if reached and t_first else 0.0,
           "unit": "x (the plain loop's first arrival at its final force residual / Newton seconds to it)",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wname, "particles": wl.n, "moving": n_moving,
                      "plain_iters": args.plain_iters, "krylov": "MINRES", "forcing": "Eisenstat-Walker 2",
                      "krylov_tol_min": 1e-4, "krylov_max": kw["krylov_max"], "move_cap": "h/4",
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
                      "vs_plain_final": (t_plain / t_newton) if reached else None,
                      "vs_plain_best": (plain[best][0] / t_best) if t_best else None},
           "device_status": rn.read_status()}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="step",
                    choices=["step", "batch", "newton", "gear", "generate", "features", "multires"])
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
    ap.add_argument("--krylov-max", type=int, default=0,
                    help="MINRES iterations per Newton step (0: the tier's default, 1 for a volume tier, "
                         "3 for a surface or feature tier: the measured best of 1-3 on the gear and the sphere)")
    ap.add_argument("--newton-tier", default="volume", choices=["volume", "surface", "feature"])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-vs-plain comparison")
    ap.add_argument("--no-secondary", action="store_true", help="skip the icosphere secondary workload")
    ap.add_argument("--cpu-sample", type=int, default=1 << 19)
    ap.add_argument("--k", type=int, default=2, help="stencil half-width of the particle cells (1 or 2)")
    ap.add_argument("--launch", default="auto",
                    help="force kernel launch shape of the timed gear tier: 'auto' (autotuned) or "
                         "'block,xcd_remap,persistent', e.g. 256,1,0 (xcd_remap 0 round-robin, "
                         "1 one contiguous range per XCD, 2 runs of 16 chunks)")
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
    if args.mode == "multires":
        return bench_multires(args)
    return bench_step(args)


def timed_steps(r, steps, warmup, label):
    """W untimed iterations, a pair-counting pass, then exactly `steps` timed
    iterations bracketed by synchronisations (HIP events on the launch stream
    around the whole region and around every force launch), then a separate
    event-timed pass for the per-phase breakdown."""
    import torch
    for _ in range(warmup):
        r.step(keep_accel=False)
    r.build_cells()
    r.accel.zero_()   # a receiver list leaves the other rows unwritten
    r.relax_step(count_pairs=True)
    r.project()
    pairs0 = float(r.accel[:, 3].double().sum().item())
    torch.cuda.synchronize()
    print(f"[bench] {label}: warmup done, {pairs0:.4g} pairs/step", file=sys.stderr, flush=True)
    r.profile(True, phases=("force",))
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        r.step(keep_accel=False)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = start.elapsed_time(stop)
    f_ms, f_n = r.profile_read()["force"]
    r.profile(True)
    for _ in range(min(steps, 50)):
        r.step(keep_accel=False)
    prof = r.profile_read()
    r.profile(False)
    r.build_cells()
    r.accel.zero_()
    r.relax_step(count_pairs=True)
    pairs1 = float(r.accel[:, 3].double().sum().item())
    print(f"[bench] {label}: {ms / steps:.4f} ms/step", file=sys.stderr, flush=True)
    return {"ms": ms, "ms_step": ms / steps, "wall": wall, "force_ms": f_ms / max(f_n, 1),
            "pairs": 0.5 * (pairs0 + pairs1), "phase_ms": {k: (v[0] / max(v[1], 1)) for k, v in prof.items() if v[1]},
            "status": r.read_status()}


def _warm_newton(rn, n_moving, kw):
    """One untimed Newton step from the start state, then the state restored:
    the solver's device vectors and snapshots are allocated (torch's caching
    allocator) before the clock starts, as the plain loop's buffers are by
    its Relaxer. The timed solve then starts from the same state."""
    import torch
    from paper_2501_03056_amd.newton import newton_relax
    snap = rn.snapshot()
    newton_relax(rn, n_moving, target=None, max_iter=1, **kw)
    rn.restore(snap)
    del snap
    torch.cuda.synchronize()


def newton_vs_plain(wl, mm, plain_iters, krylov_max, shape=None):
    """Newton-MINRES against the plain loop from the same state on one tier:
    the plain loop's residual after its iterations is the target; the
    headline ratio is the plain loop's FIRST arrival at that residual over
    Newton's time to it (its residual is not monotone). Both start with their
    device buffers allocated (the plain loop's Relaxer; one untimed Newton
    step, restored, for the solver)."""
    import torch
    from paper_2501_03056_amd import Relaxer
    from paper_2501_03056_amd.newton import newton_relax, plain_relax
    n_moving = wl.n_moving()
    rp = Relaxer(wl, device=0)
    rp.tier(mm)
    if shape:
        rp.ctx.set_launch(*shape)
    plain = plain_relax(rp, n_moving, iters=plain_iters, record_every=1)
    target, t_plain = plain[-1][1], plain[-1][0]
    t_first = _first_at_or_below(plain, target)
    best = min(range(len(plain)), key=lambda q: plain[q][1])
    del rp
    rn = Relaxer(wl, device=0)
    rn.tier(mm)
    if shape:
        rn.ctx.set_launch(*shape)
    torch.cuda.synchronize()
    kw = dict(forcing="ew", krylov_tol=1e-4, krylov_max=krylov_max, checkpoint_every=10)
    _warm_newton(rn, n_moving, kw)
    log = newton_relax(rn, n_moving, target=target, max_iter=500, time_limit=20 * t_plain + 20, **kw)
    t_newton = log.residual[-1][0]
    reached = log.residual[-1][1] <= target
    print(f"[bench] newton: R {log.residual[-1][1]:.4g} at {t_newton:.4f}s vs plain first arrival "
          f"{t_first:.4f}s, plain {plain_iters} iterations {t_plain:.4f}s", file=sys.stderr, flush=True)
    return {"metric": "Newton-HVP vs plain s to residual",
            "value": (t_first / t_newton) if reached and t_first else 0.0,
            "unit": "x (plain loop's first arrival at its final residual / Newton's seconds to it)",
            "reached": reached, "moving": n_moving, "plain_iters": plain_iters,
            "plain": {"seconds": t_plain, "R0": plain[0][1], "R_final": target,
                      "seconds_first_at_or_below_R_final": t_first, "R_best": plain[best][1],
                      "iters_to_best": best, "seconds_to_best": plain[best][0]},
            "newton_result": {"seconds": t_newton, "R": log.residual[-1][1], "newton_iters": log.newton_iters,
                              "krylov_iters": log.krylov_iters, "backtracks": log.backtracks},
            "vs_plain_final": (t_plain / t_newton) if reached else None,
            "krylov": "MINRES", "forcing": "Eisenstat-Walker 2", "krylov_max": krylov_max}


def choose_launch(args, wl):
    """The force kernel's launch shape for the timed tier: --launch B,R,P
    (threads per block, XCD remap, persistent tickets) or auto, the
    autotuner's shape search (tune.autotune at the workload's stencil, eager
    launches; 20 timed iterations per shape, cached per device in TMPDIR)."""
    from paper_2501_03056_amd.tune import autotune
    if args.launch != "auto":
        b, rm, ps = (int(v) for v in args.launch.split(","))
        return {"force_block": b, "xcd_remap": rm, "persistent": bool(ps), "source": "fixed"}
    t = autotune(wl, candidates=(args.k,), modes=("eager",), steps=20, warmup=4,
                 cache=os.path.join(os.environ.get("TMPDIR", "/tmp"), "fppg_autotune_step.json"))
    print(f"[bench] launch shapes (ms per iteration): {t['launch_ms_per_step']}", file=sys.stderr, flush=True)
    return {"force_block": t["force_block"], "xcd_remap": int(t["xcd_remap"]), "persistent": bool(t["persistent"]),
            "source": "autotuned", "ms_per_step": t["launch_ms_per_step"]}


def bench_step(args):
    import torch
    import synth
    from paper_2501_03056_amd import Relaxer

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dx = args.gear_dx
    t0 = time.perf_counter()
    wl = synth.gear_workload(dx=dx, seed=3, k=args.k)
    for g in wl.geoms:
        g.slab = args.slab
    wname = f"gear24_full_mesh_dx{dx:g}_volume_tier"
    print(f"[bench] gear dx={dx:g}: {wl.n} particles {wl.counts()} built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    mm_vol = 1 << synth.VOLUME
    wl.move_mask = mm_vol
    launch = choose_launch(args, wl)
    shape = (launch["force_block"], launch["xcd_remap"], launch["persistent"])
    r = Relaxer(wl, device=0)
    r.tier(mm_vol)
    r.ctx.set_launch(*shape)
    n_moving = r.n_moving()
    main = timed_steps(r, args.steps, args.warmup, "gear volume tier")
    ncell = int(r.geom.ncell)
    n_tri = int(r.geom.n_tri)
    del r
    # the sparse tiers of the same gear (each after the tier partition, with the receiver list)
    tiers = {}
    for name, mm in (("feature", 1 << synth.FEATURE), ("surface", 1 << synth.SURFACE)):
        wl.move_mask = mm
        rt = Relaxer(wl, device=0)
        rt.tier(mm)
        rt.use_list = True
        t = timed_steps(rt, args.tier_iters, args.warmup, f"gear {name} tier")
        tiers[name] = {"moving": rt.n_moving(), "active_particles": rt.na, "iters": args.tier_iters,
                       "ms_per_step": t["ms_step"],
                       "particle_updates_per_s": rt.n_moving() * args.tier_iters / (t["ms"] / 1e3),
                       "pairs_per_step": t["pairs"], "kernels_ms_per_step": t["phase_ms"],
                       "device_status": t["status"]}
        del rt
    tiers["volume"] = {"moving": n_moving, "ms_per_step": main["ms_step"]}
    tot_upd = sum(tiers[k]["moving"] for k in tiers) * 1.0
    tiers["three_tiers_particle_updates_per_s"] = tot_upd / sum(tiers[k]["ms_per_step"] / 1e3
                                                               for k in ("feature", "surface", "volume"))
    wl.move_mask = mm_vol
    newton = None if args.no_newton else newton_vs_plain(wl, mm_vol, args.plain_iters,
                                                         krylov_cap(args.krylov_max, "volume"), shape)
    secondary = None
    if not args.no_secondary:
        sw, sname = make_workload("sphere", args.k, args.slab)
        s_launch = choose_launch(args, sw)
        rs = Relaxer(sw, device=0)
        rs.ctx.set_launch(s_launch["force_block"], s_launch["xcd_remap"], s_launch["persistent"])
        t = timed_steps(rs, args.steps, args.warmup, "sphere")
        secondary = {"workload": sname, "particles": sw.n, "moving": sw.n_moving(),
                     "value": sw.n_moving() * args.steps / (t["ms"] / 1e3), "unit": "particle-updates/s",
                     "ms_per_step": t["ms_step"], "pair_evals_per_s": t["pairs"] * args.steps / (t["ms"] / 1e3),
                     "force_kernel_ms": t["force_ms"],
                     "force_tflops": t["pairs"] * FLOPS_PER_PAIR / (t["force_ms"] / 1e3) / 1e12,
                     "kernels_ms_per_step": t["phase_ms"], "device_status": t["status"], "force_launch": s_launch}
        del rs, sw

    ms, steps = main["ms"], args.steps
    pairs = main["pairs"]
    force_ms = main["force_ms"]
    achieved = pairs * FLOPS_PER_PAIR / (force_ms / 1e3) / 1e12
    khash = source_hash(KERNEL_SOURCES)
    launch_key = f"{shape[0]},{int(shape[1])},{int(shape[2])}"
    traffic = traffic_from_profile(khash, launch=launch_key)
    hbm = hbm_phases(wl.n, ncell, n_moving, 0, main["phase_ms"], main["ms_step"])
    out = {
        "metric": "particle-updates/s per relaxation step",
        "value": n_moving * steps / (ms / 1e3),
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "particles": wl.n, "moving": n_moving, "counts": wl.counts(),
                   "facets": n_tri, "stencil_k": int(wl.geoms[0].k), "key_slab_rows": int(args.slab),
                   "h_over_dx": 1.3, "pairs_per_step": pairs, "force_launch": launch},
        "pair_evals_per_s": pairs * steps / (ms / 1e3),
        "kernels_ms_per_step": main["phase_ms"],
        "hbm_phases": hbm,
        "roofline": {"bound": "alu", "kernel": "k_force", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "work_per_launch": pairs * FLOPS_PER_PAIR, "avg_launch_ms": force_ms,
                     "kernel_source_hash": khash, "valu_issue": valu_issue(khash, force_ms, pairs)},
        "tiers": tiers,
        "newton": newton,
        "secondary": secondary,
        "device_status": main["status"],
        "wall_s": main["wall"],
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
