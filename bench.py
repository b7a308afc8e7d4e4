"""Benchmark: multi-bounce path tracing over 2D Gaussian surfels on one GPU.

Workload (one step): a 1M-surfel 8x6x3 m room with 40 furniture boxes and
~0.5% emissive ceiling-panel surfels (scene seed 3), one 1024x768 camera at
(1.0, 3.0, 1.6) looking at (8.0, 3.0, 1.2), 64 spp, max depth 5, Russian
roulette from depth 3, 16-entry k-buffer. A step is the whole hot path on
resident inputs: BVH build over the surfels, the persistent path-tracing
kernel over all 50.3M paths, and the resolve of the fixed-point image.

Metric: ray segments traced per second (Mrays/s), counted on the device.
The roofline entry prices the path-tracing kernel by its algorithmic bytes:
68 B per blended hit (the canonical surfel record: centre, quaternion,
scales, opacity, albedo, radiance, emissive) plus 96 B of path state per
segment, over the kernel's duration from HIP events on its stream.

The CPU baseline times the FP64 brute-force oracle on a fixed sample of the
same workload's paths on the host cores.

Further workloads print their own JSON line (not the default run):
  --workload rooms5m   5M surfels in three 8x6x3 m rooms joined by doorways,
                       one 1920x1080 camera, 256 spp as 16 progressive passes
                       of 16, max depth 8, RR from 3; then an edit (radiance
                       zeroed on a random half of the emitters, albedo redrawn
                       on a random 10% of the surfels in 8 groups), a refit,
                       and the same 256 spp again.
  --workload sb100k    single-bounce reconstruction step: 100k surfels in a
                       6x4x3 m room with 12 boxes, 8 cameras at 256x256,
                       8 spp, forward render + adjoint of an L2 loss against
                       the render of a perturbed copy of the scene.
  --workload stage0    Stage-0 step: the 100k-surfel room, 8 cameras at
                       256x256; Nt, Dt, R, E render, the Eq. 4 objective
                       against a perturbed scene's images, and the adjoint
                       for every parameter.
  --workload edits     geometric edit on the 1M-surfel room: select a box
                       region, move it 1.5 m, refit; tree cost and path-
                       tracing speed (16 spp) through the refitted and a
                       rebuilt tree.
  --workload bake      light baking: the 1M-surfel room with half its
                       emitters off, path-traced targets of 8 interior views
                       at 512x384 (64 spp, depth 5), one bake iteration
                       (0-bounce render, PQ-L1 loss, radiance gradient, Adam)
                       per step.
  --workload mis       emitter sampling (selection by 1 m cells; --mis-cell 0
                       selects by power) combined with cosine sampling by
                       multiple importance sampling on the default room:
                       time per 64-spp image and image error of it and of
                       the plain path tracer against a reference of 8x the
                       spp (512), at equal spp and at equal time
                       (--mis-config 4: the three-room 5M scene at 64 spp).
  --workload serve     continuous-batching server against one-at-a-time FIFO
                       on the same Poisson arrivals over a resident 3M-surfel
                       room (request mix scaled down by default: 128x128 or
                       256x256, 4 or 16 spp, 5% edits; --mix full takes the
                       configuration's 256^2..1920x1080 and 16..256 spp), at
                       0.5, 0.8 and 0.95 of the FIFO service rate; latency
                       percentiles per load.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--workload room1m|rooms5m|sb100k|stage0|bake|edits|mis|serve]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0
PROFILE = os.path.join(HERE, "profiles", "k_path_trace_room1m_1024x768_64spp.md")
ALGO_BYTES_PER_HIT = 68
ALGO_BYTES_PER_SEGMENT = 96


def _log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _oracle_worker(args):
    import oracle.render as R
    pixels, samples = args
    t0 = time.perf_counter()
    out = R.path_trace(_ORACLE["sc"], _ORACLE["cam"], _ORACLE["prm"], pixels=pixels, samples=samples)
    return int(out["nseg"].sum()), time.perf_counter() - t0


_ORACLE = {}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(scene, cam, params, full_segments, budget_paths=1024):
    """Oracle segments/s on a fixed sample of the workload's paths, across
    the host cores this process may use (at most 16, the host's share per
    GPU) with a fork pool, and the time the oracle would take for the whole
    workload at that rate (extrapolated, not run)."""
    import multiprocessing as mp

    from oracle import Params
    from oracle.tracer import Scene64
    prm = Params(spp=params.spp, max_depth=params.max_depth, rr_start=params.rr_start, seed=params.seed,
                 camera_id=params.camera_id)
    _ORACLE.update(sc=Scene64(scene), cam=cam, prm=prm)
    rng = np.random.default_rng(7)
    pix = rng.choice(cam.width * cam.height, budget_paths, replace=False)
    samp = rng.integers(0, params.spp, budget_paths)
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    cores = min(usable, 16, budget_paths)
    jobs = [(np.array([p]), [int(s)]) for p, s in zip(pix, samp)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    segs = sum(r[0] for r in res)
    rate = segs / wall
    return {"value": rate / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"{budget_paths} random (pixel, sample) paths of the same frame, {segs} segments, "
                      f"{wall:.1f} s wall on {cores} processes",
            "host": {"os_cpu_count": os.cpu_count(), "usable_cpus": usable, "cpu_model": _cpu_model()},
            "extrapolated_full_workload_s": round(full_segments / rate, 1),
            "extrapolated_note": f"extrapolated, not run: the workload's {int(full_segments)} segments per step "
                                 f"at the sampled oracle rate on {cores} processes"}


def copy_calibration(torch, mib):
    """A plain device copy (read n bytes, write n bytes) through torch's
    elementwise kernel, to scale the HBM byte counters of the other kernels."""
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 3}))

def _code_tokens(text):
    """Source text without C/C++ comments and with whitespace collapsed, so
    that only code changes alter the hash."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


# what the path-tracing kernel is compiled from, and the BVH build it traverses
KERNEL_SOURCES = ["paper_2601_23065_amd/csrc/eag_pt.hip", "paper_2601_23065_amd/csrc/eag_build.hip",
                  "paper_2601_23065_amd/csrc/eag_prim.hip", "paper_2601_23065_amd/csrc/eag_runner.h",
                  "paper_2601_23065_amd/csrc/eag_device.h", "paper_2601_23065_amd/csrc/eag_render.h",
                  "paper_2601_23065_amd/csrc/eag_internal.h", "include/eag.h", "paper_2601_23065_amd/build.py"]


def kernel_source_hash():
    """sha256 over the code the path-tracing kernel is compiled from
    (relative names and comment-free contents, in a fixed order)."""
    h = hashlib.sha256()
    files = [os.path.join(HERE, f) for f in KERNEL_SOURCES]
    for f in files:
        h.update(os.path.relpath(f, HERE).encode())
        with open(f, encoding="utf-8") as fh:
            h.update(_code_tokens(fh.read()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the path-tracing kernel on the default
    workload, from the committed counter profile (FETCH_SIZE and WRITE_SIZE,
    each scaled by a copy kernel's reading); None when the kernel sources
    have changed since the counters were taken."""
    try:
        with open(PROFILE) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines() if ": " in line)
    except OSError:
        return None
    if kv.get("source_sha256") != kernel_source_hash() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def _roofline(blended, segments, pt_ms):
    algo_bytes = blended * ALGO_BYTES_PER_HIT + segments * ALGO_BYTES_PER_SEGMENT
    achieved = algo_bytes / (pt_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": None}


def bench_rooms5m(torch, args):
    """Progressive rendering of the three-room scene, an edit, a refit, and
    the same render again (one JSON line)."""
    import scenegen as sg
    from paper_2601_23065_amd import EDIT_SET_ALBEDO, EDIT_SET_RADIANCE
    from paper_2601_23065_amd.api import BVH, Params, Scene, apply_edit, path_trace, path_trace_workspace, resolve

    scene, cams, cfg = sg.config(4, n_override=args.surfels)
    cam = cams[0]
    spp, pass_spp = args.spp or cfg["spp"], cfg["pass_spp"]
    params = Params(spp=spp, max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=0)
    _log(f"scene ready: {scene.n} surfels, {cam.width}x{cam.height}, {spp} spp in passes of {pass_spp}")
    gs = Scene(scene.arrays())
    ws = path_trace_workspace(gs)
    counters = torch.zeros(6, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    eb0 = ev()
    bvh = BVH(gs)
    eb1 = ev()

    def render(tag):
        acc, evs = None, []
        for s0 in range(0, spp, pass_spp):
            a = ev()
            acc = path_trace(bvh, gs, cam, params, s0, min(pass_spp, spp - s0), accum=acc, counters=counters, ws=ws)
            evs.append((a, ev()))
        img = resolve(acc, spp)
        torch.cuda.synchronize()
        passes = [a.elapsed_time(b) for a, b in evs]
        _log(f"{tag}: {len(passes)} passes, {sum(passes):.0f} ms")
        return img, passes

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    img0, passes0 = render("before the edit")
    rng = np.random.default_rng(4)
    emit = np.nonzero(scene.emissive > 0)[0]
    off = np.sort(rng.choice(emit, emit.size // 2, replace=False)).astype(np.int32)
    groups = np.array_split(np.sort(rng.choice(scene.n, scene.n // 10, replace=False)).astype(np.int32), 8)
    colors = [tuple(map(float, rng.uniform(0.05, 0.9, 3))) for _ in groups]
    off_d = torch.from_numpy(off).cuda()
    groups_d = [torch.from_numpy(g).cuda() for g in groups]
    ee0 = ev()
    apply_edit(gs, EDIT_SET_RADIANCE, off_d, (0.0, 0.0, 0.0))
    for g, c in zip(groups_d, colors):
        apply_edit(gs, EDIT_SET_ALBEDO, g, c)
    ee1 = ev()
    bvh.refit(gs)
    ee2 = ev()
    img1, passes1 = render("after the edit")
    wall = time.perf_counter() - t0
    c = counters.cpu().numpy().astype(np.float64)
    segments, paths, rounds, tests, blended, visits = c
    pt_ms = sum(passes0) + sum(passes1)
    rec = {
        "metric": "Mrays/s multi-bounce PT over 2D Gaussians",
        "value": round(segments / wall / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": 2,
        "warmup": 0,
        "ms_per_step": round(wall / 2 * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"progressive path tracing, {scene.n} surfels in three 8x6x3 m rooms joined by "
                               f"doorways, {cam.width}x{cam.height}, {spp} spp in passes of {pass_spp}, max depth "
                               f"{params.max_depth}, RR from {params.rr_start}; step = one full render; between the "
                               f"two steps: radiance edit on half the emitters, albedo edit on 10% of the surfels, "
                               f"refit",
                   "surfels": scene.n, "width": cam.width, "height": cam.height, "spp": spp,
                   "max_depth": params.max_depth},
        "roofline": _roofline(blended, segments, pt_ms),
        "detail": {"segments": segments, "paths": paths, "kbuf_rounds_per_segment": round(rounds / segments, 3),
                   "candidate_tests_per_segment": round(tests / segments, 2),
                   "nodes_visited_per_segment": round(visits / segments, 2),
                   "blended_hits_per_segment": round(blended / segments, 3),
                   "bvh_build_ms": round(eb0.elapsed_time(eb1), 3),
                   "pass_ms_before": [round(x, 1) for x in passes0], "pass_ms_after": [round(x, 1) for x in passes1],
                   "edit_ms": round(ee0.elapsed_time(ee1), 3), "refit_ms": round(ee1.elapsed_time(ee2), 3),
                   "emitters_zeroed": int(off.size), "surfels_recoloured": int(sum(g.size for g in groups)),
                   "image_mean_before": float(img0.mean()), "image_mean_after": float(img1.mean())},
    }
    print(json.dumps(rec))

def bench_sb100k(torch, args):
    """Single-bounce reconstruction step on the 100k-surfel room (one JSON
    line): forward render of 8 cameras, then the adjoint of an L2 loss
    against the render of a perturbed copy of the scene."""
    import scenegen as sg
    from paper_2601_23065_amd.api import BVH, Params, Scene, SingleBounceRender, render_single_bounce

    scene, cams, cfg = sg.config(2, n_override=args.surfels)
    p = Params(spp=args.spp or cfg["spp"], seed=0)
    tgt = sg.perturb(scene)
    gt = Scene(tgt.arrays())
    target = render_single_bounce(BVH(gt), gt, cams, p)
    gs = Scene(scene.arrays())
    bvh = BVH(gs)
    leaves = {k: getattr(gs, k).clone().requires_grad_(k != "emissive")
              for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance", "emissive")}
    # rays of one forward: a camera segment per pixel, spp secondary segments per reflecting pixel
    _, state = render_single_bounce(bvh, gs, cams, p, keep_state=True)
    npix = len(cams) * cams[0].width * cams[0].height
    reflect = int((state[:npix * 28].view(npix, 28)[:, 25] == 2.0).sum())
    rays = npix + reflect * p.spp
    _log(f"scene ready: {scene.n} surfels, {len(cams)} cameras {cams[0].width}x{cams[0].height}, {p.spp} spp, "
         f"{rays} segments per forward")
    stream = torch.cuda.current_stream()

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for v in leaves.values():
            v.grad = None
        e[0].record(stream)
        rgb = SingleBounceRender.apply(*leaves.values(), bvh, gs, cams, p)
        e[1].record(stream)
        loss = ((rgb - target) ** 2).sum()
        loss.backward()
        e[2].record(stream)
        return e

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = float(np.mean([a.elapsed_time(b) for a, b, _ in evs]))
    bwd = float(np.mean([b.elapsed_time(c) for _, b, c in evs]))
    gnorm = {k: float(v.grad.norm()) for k, v in leaves.items() if v.grad is not None}
    rec = {
        "metric": "Mrays/s single-bounce forward (segments traced per second)",
        "value": round(rays / (fwd * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single-bounce reconstruction step, {scene.n} surfels in a 6x4x3 m room with 12 "
                               f"boxes, {len(cams)} cameras {cams[0].width}x{cams[0].height}, {p.spp} spp; step = "
                               f"forward render + adjoint of an L2 loss against a perturbed scene's render",
                   "surfels": scene.n, "cameras": len(cams), "width": cams[0].width, "height": cams[0].height,
                   "spp": p.spp},
        "detail": {"forward_ms": round(fwd, 3), "backward_ms": round(bwd, 3), "segments_per_forward": rays,
                   "backward_Mrays_per_s": round(rays / (bwd * 1e-3) / 1e6, 3), "grad_norms": gnorm},
    }
    print(json.dumps(rec))



def bench_edits(torch, args):
    """Geometric edit on the 1M-surfel room (one JSON line): select the
    surfels of a box region (a corner of the room with its furniture), move
    them 1.5 m, then refit the tree and, separately, rebuild it; the tree
    cost of both and path-tracing speed (1024x768, 16 spp) through both."""
    import scenegen as sg
    from paper_2601_23065_amd.api import (BVH, Params, Scene, move_surfels, path_trace, path_trace_workspace,
                                          select_box)

    scene, cams, cfg = sg.config(3, n_override=args.surfels)
    cam = cams[0]
    gs = Scene(scene.arrays())
    bvh = BVH(gs)
    ws = path_trace_workspace(gs)
    stream = torch.cuda.current_stream()

    def timed(f):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = f()
        b.record(stream)
        torch.cuda.synchronize()
        return out, a.elapsed_time(b)

    cost0 = float(bvh.cost_at_build)
    idx, sel_ms = timed(lambda: select_box(gs, (0.0, 0.0, 0.0), (3.0, 3.0, 3.0)))
    _, move_ms = timed(lambda: move_surfels(gs, idx, t=(1.5, 0.0, 0.0)))
    _, refit_ms = timed(lambda: bvh.refit(gs))
    cost_refit = float(bvh.sah_cost())
    fresh, build_ms = timed(lambda: BVH(gs))
    cost_fresh = float(fresh.cost_at_build)
    p = Params(spp=args.spp or 16, max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0)
    counters = torch.zeros(6, dtype=torch.int64, device="cuda")

    def pt(tree):
        counters.zero_()
        path_trace(tree, gs, cam, p, 0, p.spp, counters=counters, ws=ws)   # warm-up
        counters.zero_()
        _, ms = timed(lambda: path_trace(tree, gs, cam, p, 0, p.spp, counters=counters, ws=ws))
        return float(counters[0]) / (ms * 1e-3) / 1e6, ms

    rate_refit, ms_refit = pt(bvh)
    rate_fresh, ms_fresh = pt(fresh)
    rec = {
        "metric": "path-tracing Mrays/s through the refitted tree after a geometric edit",
        "value": round(rate_refit, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(sel_ms + move_ms + refit_ms + ms_refit, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"geometric edit, {scene.n} surfels in an 8x6x3 m room with 40 boxes: the "
                               f"{int(idx.numel())} surfels in the box [0,3]^3 moved 1.5 m along x; step = select + "
                               f"move + refit + path tracing {cam.width}x{cam.height} at {p.spp} spp",
                   "surfels": scene.n, "moved": int(idx.numel()), "spp": p.spp},
        "detail": {"select_ms": round(sel_ms, 3), "move_ms": round(move_ms, 3), "refit_ms": round(refit_ms, 3),
                   "rebuild_ms": round(build_ms, 3), "cost_at_build": round(cost0, 4),
                   "cost_refitted": round(cost_refit, 4), "cost_rebuilt": round(cost_fresh, 4),
                   "pt_ms_refitted": round(ms_refit, 3), "pt_ms_rebuilt": round(ms_fresh, 3),
                   "Mrays_per_s_rebuilt": round(rate_fresh, 3)},
    }
    print(json.dumps(rec))


def bench_stage0(torch, args):
    """Stage-0 step (one JSON line): the 100k-surfel room, 8 cameras at
    256x256; targets are the Stage-0 images of a perturbed copy of the scene
    (its R as the colour target, its Nt as the monocular normals, E > tau_E
    as the emission mask); a step renders Nt, Dt, R, E, evaluates Eq. 4 with
    unit weights and runs the adjoint for every parameter."""
    import scenegen as sg
    from paper_2601_23065_amd.api import BVH, Params, Scene, render_stage0, stage0_backward, stage0_loss

    scene, cams, cfg = sg.config(2, n_override=args.surfels)
    p = Params(spp=1, seed=0)
    tgt = sg.perturb(scene)
    gt = Scene(tgt.arrays())
    ti, _ = render_stage0(BVH(gt), gt, cams, p)
    rgb_gt = ti[..., 4:7].contiguous()
    n_mono = ti[..., 0:3].contiguous()
    mask = (ti[..., 7:8] > p.tau_E).float().contiguous()
    gs = Scene(scene.arrays())
    bvh = BVH(gs)
    npix = len(cams) * cams[0].width * cams[0].height
    _log(f"scene ready: {scene.n} surfels, {len(cams)} cameras {cams[0].width}x{cams[0].height}")
    stream = torch.cuda.current_stream()
    grads = {k: torch.zeros_like(gs.t[k]) for k in ("pos", "rot", "scale", "opacity", "radiance", "emissive")}

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for v in grads.values():
            v.zero_()
        e[0].record(stream)
        images, state = render_stage0(bvh, gs, cams, p)
        e[1].record(stream)
        loss, d = stage0_loss(images, rgb_gt, n_mono, mask, cams, p)
        e[2].record(stream)
        stage0_backward(bvh, gs, cams, p, d, state, grads)
        e[3].record(stream)
        return e, loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = float(np.mean([e[0].elapsed_time(e[1]) for e, _ in evs]))
    lss = float(np.mean([e[1].elapsed_time(e[2]) for e, _ in evs]))
    bwd = float(np.mean([e[2].elapsed_time(e[3]) for e, _ in evs]))
    tot = float(np.mean([e[0].elapsed_time(e[3]) for e, _ in evs]))
    rec = {
        "metric": "Stage-0 steps per second",
        "value": round(1e3 / tot, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Stage-0 step, {scene.n} surfels in a 6x4x3 m room with 12 boxes, {len(cams)} cameras "
                               f"{cams[0].width}x{cams[0].height}; step = Nt, Dt, R, E render + Eq. 4 (PQ-L1, normal, "
                               f"distance normal, emission; unit weights) + adjoint for every parameter, against a "
                               f"perturbed scene's images",
                   "surfels": scene.n, "cameras": len(cams), "width": cams[0].width, "height": cams[0].height},
        "detail": {"render_ms": round(fwd, 3), "loss_ms": round(lss, 3), "backward_ms": round(bwd, 3),
                   "camera_rays_per_step": 2 * npix, "Mrays_per_s": round(2 * npix / (tot * 1e-3) / 1e6, 3),
                   "loss": float(evs[-1][1]),
                   "grad_norms": {k: float(v.norm()) for k, v in grads.items()}},
    }
    print(json.dumps(rec))


def bench_bake(torch, args):
    """Light baking (one JSON line): the 1M-surfel room with half of its
    emitters switched off, path-traced targets (64 spp, depth 5, RR from 3)
    for 8 interior views at 512x384, then bake iterations of the radiance
    into the 0-bounce image starting from the unedited radiance; a step is
    one iteration (render, PQ-L1 loss, radiance gradient, Adam update)."""
    import scenegen as sg
    from paper_2601_23065_amd import EDIT_SET_RADIANCE
    from paper_2601_23065_amd.api import Adam, Baker, BVH, Params, Scene, apply_edit, path_trace, resolve

    scene, _, cfg = sg.config(3, n_override=args.surfels)
    cams = sg.interior_cameras(scene, 8, 512, 384, seed=21)
    gs = Scene(scene.arrays())
    bvh = BVH(gs)
    emit = np.nonzero(scene.emissive > 0)[0]
    off = np.sort(np.random.default_rng(5).choice(emit, emit.size // 2, replace=False)).astype(np.int32)
    r0 = gs.t["radiance"].clone()
    apply_edit(gs, EDIT_SET_RADIANCE, torch.from_numpy(off).cuda(), (0.0, 0.0, 0.0))
    pt = Params(spp=args.spp or cfg["spp"], max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=1)
    tg = []
    for ci, cam in enumerate(cams):
        pt.camera_id = ci
        tg.append(resolve(path_trace(bvh, gs, cam, pt), pt.spp))
    targets = torch.stack(tg)
    gs.t["radiance"].copy_(r0)
    baker = Baker(bvh, gs, cams, Params(spp=1), targets, Adam(lr=0.05))
    npix = len(cams) * cams[0].width * cams[0].height
    _log(f"targets ready: {scene.n} surfels, {len(cams)} views {cams[0].width}x{cams[0].height}, {pt.spp} spp")
    stream = torch.cuda.current_stream()
    losses = []
    for _ in range(args.warmup):
        losses.append(float(baker.step()))
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        loss = baker.step()
        b.record(stream)
        evs.append((a, b, loss.clone()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = float(np.mean([a.elapsed_time(b) for a, b, _ in evs]))
    losses += [float(l) for _, _, l in evs]
    rec = {
        "metric": "light-baking iterations per second",
        "value": round(1e3 / ms, 3),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"light baking, {scene.n} surfels in an 8x6x3 m room with 40 boxes, half the emitters "
                               f"off, path-traced targets ({pt.spp} spp, depth {pt.max_depth}) of {len(cams)} views "
                               f"{cams[0].width}x{cams[0].height}; step = 0-bounce render + PQ-L1 loss + radiance "
                               f"gradient + Adam update",
                   "surfels": scene.n, "views": len(cams), "width": cams[0].width, "height": cams[0].height},
        "detail": {"iteration_ms": round(ms, 3), "camera_rays_per_iteration": 2 * npix,
                   "Mrays_per_s": round(2 * npix / (ms * 1e-3) / 1e6, 3),
                   "loss_first": losses[0], "loss_last": losses[-1]},
    }
    print(json.dumps(rec))


def bench_mis(torch, args):
    """Emitter sampling with multiple importance sampling against the plain
    path tracer on the benchmark room: time per 64-spp image and image error
    against a converged reference at equal spp and at equal time (one JSON
    line)."""
    import scenegen as sg
    from paper_2601_23065_amd.api import (BVH, Emitters, Params, Scene, path_trace, path_trace_mis,
                                          path_trace_mis_workspace, path_trace_workspace)

    scene, cams, cfg = sg.config(args.mis_config, n_override=args.surfels)
    cam = cams[0]
    spp = args.spp or (64 if args.mis_config == 4 else cfg["spp"])
    params = Params(spp=spp, max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=0)
    gs = Scene(scene.arrays())
    ws = path_trace_workspace(gs)
    ws_mis = path_trace_mis_workspace(gs, cam, params)
    stream = torch.cuda.current_stream()
    bvh = BVH(gs)
    te0 = time.perf_counter()
    em = Emitters(gs, params, cell=args.mis_cell)
    table_ms = (time.perf_counter() - te0) * 1e3
    n_em, _ = em.info()
    _log(f"scene ready: {scene.n} surfels, {n_em} emitters, {cam.width}x{cam.height}, {spp} spp")
    counters = torch.zeros(7, dtype=torch.int64, device="cuda")

    def image(fn, s0, count):
        acc = fn(s0, count)
        return acc.double() / (2.0 ** 32 * count)

    def mis(s0, count, c=None):
        return path_trace_mis(bvh, gs, em, cam, params, s0, count, counters=c, ws=ws_mis)

    def plain(s0, count, c=None):
        return path_trace(bvh, gs, cam, params, s0, count, counters=c, ws=ws)

    # converged reference: 8x the spp (512 at 64 spp) of the emitter-sampled estimator on sample indices
    # disjoint from the tests
    ref = None
    per = max(1, spp // 2)
    for k in range(16):
        a = image(mis, 100000 + per * k, per)
        ref = a if ref is None else ref + a
        torch.cuda.synchronize()
        _log(f"reference pass {k + 1}/16")
    ref /= 16

    def timed(fn):
        for _ in range(args.warmup):
            fn(0, spp)
        torch.cuda.synchronize()
        counters.zero_()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            acc = fn(0, spp, counters)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps * 1e3
        c = counters.cpu().numpy().astype(np.float64) / args.steps
        img = acc.double() / (2.0 ** 32 * spp)
        rmse = float(torch.sqrt(((img - ref) ** 2).mean()))
        return wall, ev0.elapsed_time(ev1) / args.steps, c, rmse

    ms_mis, kms_mis, c_mis, rmse_mis = timed(mis)
    _log("emitter-sampled timing done")
    ms_plain, kms_plain, c_plain, rmse_plain = timed(plain)
    _log("plain timing done")
    segments, paths, rounds, tests, blended, visits, dropped = c_mis
    assert dropped == 0, f"{dropped} light-pdf queue entries dropped"
    value = segments / (ms_mis * 1e-3) / 1e6
    rec = {
        "metric": "Mrays/s multi-bounce PT over 2D Gaussians with emitter sampling + MIS",
        "value": round(value, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_mis, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"path tracing with emitter sampling and MIS (power heuristic; selection "
                               + (f"by {args.mis_cell} m cells" if args.mis_cell > 0 else "by power")
                               + f"), {scene.n} surfels "
                               f"({n_em} emitters) in " + ("three 8x6x3 m rooms joined by doorways, 120 boxes"
                                                           if args.mis_config == 4 else "an 8x6x3 m room with 40 boxes")
                               + f", {cam.width}x{cam.height}, "
                               f"{spp} spp, max depth {params.max_depth}, RR from {params.rr_start}; step = the "
                               f"path-tracing launch over all samples",
                   "surfels": scene.n, "emitters": n_em, "width": cam.width, "height": cam.height, "spp": spp,
                   "selection_cell": args.mis_cell},
        "roofline": _roofline(blended, segments, kms_mis),
        "detail": {"segments_per_step": segments, "paths_per_step": paths,
                   "light_pdf_note": "segments include one light segment per reflecting vertex whose sample "
                                     "lies above the surface",
                   "mis_image_ms": round(ms_mis, 3), "plain_image_ms": round(ms_plain, 3),
                   "plain_segments_per_step": c_plain[0], "plain_mrays_s": round(c_plain[0] / (ms_plain * 1e-3) / 1e6, 3),
                   "per_segment_mis": {k: round(v / max(segments, 1), 3) for k, v in
                                       zip(("rounds", "tests", "blended", "visits"), (rounds, tests, blended, visits))},
                   "per_segment_plain": {k: round(v / max(c_plain[0], 1), 3) for k, v in
                                         zip(("rounds", "tests", "blended", "visits"), c_plain[2:6])},
                   "light_pdf_queue_dropped": int(dropped),
                   "rmse_mis": rmse_mis, "rmse_plain": rmse_plain,
                   "mse_ratio_equal_spp": round((rmse_plain / rmse_mis) ** 2, 3),
                   "mse_ratio_equal_time": round((rmse_plain / rmse_mis) ** 2 * ms_plain / ms_mis, 3),
                   "emitter_table_ms": round(table_ms, 3),
                   "reference": f"{16 * per} spp of the emitter-sampled estimator on disjoint sample indices"},
    }
    print(json.dumps(rec))


def bench_serve(torch, args):
    """Continuous batching against FIFO on the same arrivals (one JSON line)."""
    import scenegen as sg
    from paper_2601_23065_amd import EDIT_SCALE_RADIANCE, EDIT_SET_ALBEDO
    from paper_2601_23065_amd.api import BVH, Params, Scene, Server, apply_edit, path_trace, resolve

    scene, _, cfg = sg.config(5, n_override=args.surfels)
    n_req = args.requests
    if args.mix == "full":
        mix = dict(resolutions=((256, 256), (512, 512), (1024, 768), (1920, 1080)), spps=(16, 64, 256))
    else:
        mix = dict(resolutions=((128, 128), (256, 256)), spps=(4, 16))
    kinds = {"scale_radiance": EDIT_SCALE_RADIANCE, "set_albedo": EDIT_SET_ALBEDO}
    _log(f"scene ready: {scene.n} surfels, {n_req} requests per run")

    def params_of(i, r):
        return Params(spp=r["spp"], max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=i)

    def fifo(reqs, realtime, keep=False):
        """One request at a time through the plain path tracer, in arrival
        order; returns latencies (or service times) in s, and the images
        when keep."""
        gs = Scene(scene.arrays())
        bvh = BVH(gs)
        torch.cuda.synchronize()
        out = []
        images = []
        t_start = time.perf_counter()
        for i, r in enumerate(reqs):
            if realtime:
                delay = t_start + r["t"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            t_req = time.perf_counter()
            if r["kind"] == "edit":
                apply_edit(gs, kinds[r["op"]], torch.from_numpy(r["idx"]).cuda(), r["value"])
                continue
            acc = path_trace(bvh, gs, r["camera"], params_of(i, r))
            img = resolve(acc, r["spp"])
            torch.cuda.synchronize()
            done = time.perf_counter()
            out.append(done - (t_start + r["t"]) if realtime else done - t_req)
            if keep:
                images.append(img)
            _log(f"fifo: {i + 1} of {len(reqs)} requests ({r['camera'].width}x{r['camera'].height}, {r['spp']} spp)")
        out = np.array(out)
        return (out, images) if keep else out

    def batched(reqs, keep=False):
        gs = Scene(scene.arrays())
        need = L_arena(scene.n)
        srv = Server(gs, arena_bytes=need, max_live_requests=8,
                     paths_per_launch=(1 << 22) if args.mix == "full" else (1 << 20))
        tickets = []
        t_start = time.perf_counter()
        for i, r in enumerate(reqs):
            delay = t_start + r["t"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            if r["kind"] == "edit":
                srv.edit(kinds[r["op"]], r["idx"], r["value"])
            else:
                tickets.append(srv.submit(r["camera"], params_of(i, r)))
            _log(f"batched: {i + 1} of {len(reqs)} requests submitted")
        _log("batched: all requests submitted")
        lat = []
        for k, (t, img) in enumerate(tickets):
            res = srv.wait(t, timeout=1200.0)
            assert res["status"] == 0, res
            lat.append(res["t_done"] - res["t_submit"])
            _log(f"batched: {k + 1} of {len(tickets)} requests done")
        srv.close()
        lat = np.array(lat)
        return (lat, [img for _, img in tickets]) if keep else lat

    def L_arena(n):
        from paper_2601_23065_amd import _lib
        w, h = max(mix["resolutions"], key=lambda r: r[0] * r[1])
        return int(_lib.load().eag_serve_arena_bytes(n, 3, 8 * w * h * 24)) + (64 << 20)

    cal = sg.arrivals(scene, n_req, 1.0, **mix)
    fifo(cal[:2], False)   # warm-up: code objects, allocator
    if args.serve_rate > 0:
        mu = args.serve_rate
        service = np.array([1.0 / mu])
        _log(f"FIFO service rate given: {mu:.4f} requests/s")
    else:
        service = fifo(cal, False)
        mu = service.size / service.sum()
        _log(f"FIFO service rate {mu:.4f} requests/s (mean {service.mean() * 1e3:.1f} ms over {service.size})")
    loads = {}
    identical = {}
    for rho in (float(x) for x in args.serve_loads.split(",") if x):
        reqs = sg.arrivals(scene, n_req, rho * mu, **mix)
        lf, imf = fifo(reqs, True, keep=True)
        lb, imb = batched(reqs, keep=True)
        identical[str(rho)] = all(torch.equal(a, b) for a, b in zip(imf, imb)) and len(imf) == len(imb)
        del imf, imb
        loads[str(rho)] = {k: {"p50_ms": round(float(np.percentile(v, 50)) * 1e3, 2),
                               "p99_ms": round(float(np.percentile(v, 99)) * 1e3, 2),
                               "mean_ms": round(float(v.mean()) * 1e3, 2)} for k, v in (("batched", lb), ("fifo", lf))}
        _log(f"load {rho}: {loads[str(rho)]}; served images equal FIFO's: {identical[str(rho)]}")
    errors = serve_oracle_check(torch, scene, cfg, mix, args) if args.serve_check else None
    key = "0.8" if "0.8" in loads else (next(iter(loads)) if loads else None)
    rec = {
        "metric": f"p99 request latency at {key} load, continuous batching",
        "value": loads[key]["batched"]["p99_ms"] if key else None,
        "unit": "ms",
        "n_gpus": 1,
        "steps": n_req,
        "warmup": 4,
        "ms_per_step": round(1e3 / mu, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"render server over a resident {scene.n}-surfel 8x6x3 m room, Poisson arrivals of "
                               f"{n_req} requests per load (resolutions {mix['resolutions']}, spp {mix['spps']}, "
                               f"depth 5, 5% attribute edits) at {args.serve_loads} of the FIFO service rate",
                   "surfels": scene.n, "requests": n_req, "mix": args.mix},
        "detail": {"fifo_service_rate_per_s": round(mu, 4), "fifo_mean_service_ms": round(service.mean() * 1e3, 3),
                   "service_rate_measured": args.serve_rate <= 0, "loads": loads,
                   "served_images_equal_fifo": identical, "oracle_error_per_class": errors},
    }
    print(json.dumps(rec))



def _serve_oracle_job(args):
    import oracle.render as R
    k, cam, prm, pixels, sample = args
    out = R.path_trace(_ORACLE["sc"], cam, prm, pixels=pixels, samples=[sample])
    return k, out["value"][:, 0], out["flags"][:, 0]


def serve_oracle_check(torch, scene, cfg, mix, args, per_class=256):
    """Image error against the oracle for each request class of the mix
    (resolution x spp): a request of the class (camera and parameters as the
    served ones) renders one of its samples alone through the same kernel,
    and per_class seeded pixels of that sample are compared path by path
    with the oracle (the served image is a fixed-point sum of such paths,
    identical whether served in a mix or alone). Max relative error over
    unflagged paths, |a - b| / max(|b|, 1e-2 RMS(b))."""
    import multiprocessing as mp

    import scenegen as sg
    from oracle import Params as OParams
    from oracle.tracer import Scene64
    from paper_2601_23065_amd.api import BVH, Params, Scene, path_trace
    gs = Scene(scene.arrays())
    bvh = BVH(gs)
    cams = sg.interior_cameras(scene, len(mix["resolutions"]) * len(mix["spps"]), 16, 16, seed=606)
    rng = np.random.default_rng(607)
    jobs, gpu = [], {}
    k = 0
    for (w, h) in mix["resolutions"]:
        for spp in mix["spps"]:
            c = cams[k]
            cam = sg.Camera(c.eye, c.look_at, c.up, c.vfov_deg, w, h)
            p = Params(spp=spp, max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=1000 + k)
            sample = int(rng.integers(spp))
            acc = path_trace(bvh, gs, cam, p, sample, 1)
            pix = np.sort(rng.choice(w * h, per_class, replace=False))
            gpu[k] = (f"{w}x{h} {spp} spp", acc.cpu().numpy().reshape(-1, 3)[pix].astype(np.float64) / 2.0 ** 32)
            prm = OParams(spp=spp, max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=1000 + k)
            jobs += [(k, cam, prm, pix[i:i + 16], sample) for i in range(0, per_class, 16)]
            k += 1
    _log(f"serve oracle check: {len(jobs)} jobs of 16 paths")
    _ORACLE.update(sc=Scene64(scene))
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    with mp.get_context("fork").Pool(min(usable, 16)) as pool:
        res = pool.map(_serve_oracle_job, jobs, chunksize=1)
    out = {}
    for kk, (name, got) in gpu.items():
        ref = np.concatenate([v for j, v, f in res if j == kk])
        flags = np.concatenate([f for j, v, f in res if j == kk])
        ok = flags == 0
        a, b = got[ok], ref[ok]
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        err = np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-30)
        out[name] = {"paths": int(ok.size), "unflagged": int(ok.sum()), "nonzero": int(np.count_nonzero(b.sum(1))),
                     "max_rel_err": float(err.max()) if err.size else None}
        _log(f"serve oracle check {name}: {out[name]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--surfels", type=int, default=None, help="override the workload's surfel count")
    ap.add_argument("--requests", type=int, default=100, help="requests per run of the serve workload")
    ap.add_argument("--mix", default="small", choices=["small", "full"],
                    help="serve workload request mix: small (128^2 or 256^2, 4 or 16 spp) or full "
                         "(256^2 .. 1920x1080, 16 .. 256 spp)")
    ap.add_argument("--spp", type=int, default=None, help="override the workload's 64 spp (diagnostics only)")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95", help="serve workload: loads to run (fractions of the "
                    "FIFO service rate)")
    ap.add_argument("--serve-rate", type=float, default=0.0, help="serve workload: FIFO service rate (requests/s) "
                    "from an earlier calibration; 0 measures it")
    ap.add_argument("--serve-check", action="store_true", help="serve workload: image error of each request class "
                    "against the oracle (host cores)")
    ap.add_argument("--mis-config", type=int, default=3, choices=[3, 4],
                    help="scene of the mis workload: 3 = the default room, 4 = the three rooms (64 spp)")
    ap.add_argument("--mis-cell", type=float, default=1.0,
                    help="emitter selection of the mis workload: 0 = by power, a power of two = by cells of that size")
    ap.add_argument("--workload", default="room1m",
                    choices=["room1m", "rooms5m", "serve", "sb100k", "bake", "stage0", "edits", "mis"])
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run an elementwise copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calib:
        copy_calibration(torch, args.copy_calib)
        return
    if args.workload == "rooms5m":
        bench_rooms5m(torch, args)
        return
    if args.workload == "serve":
        bench_serve(torch, args)
        return
    if args.workload == "sb100k":
        bench_sb100k(torch, args)
        return
    if args.workload == "bake":
        bench_bake(torch, args)
        return
    if args.workload == "stage0":
        bench_stage0(torch, args)
        return
    if args.workload == "edits":
        bench_edits(torch, args)
        return
    if args.workload == "mis":
        bench_mis(torch, args)
        return

    import scenegen as sg
    from paper_2601_23065_amd.api import BVH, Params, Scene, path_trace, path_trace_workspace, resolve

    scene, cams, cfg = sg.config(3, n_override=args.surfels)
    cam = cams[0]
    params = Params(spp=args.spp or cfg["spp"], max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0,
                    camera_id=0)
    _log(f"scene ready: {scene.n} surfels, {cam.width}x{cam.height}, {params.spp} spp")
    gs = Scene(scene.arrays())
    ws = path_trace_workspace(gs)
    counters = torch.zeros(6, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        evb = torch.cuda.Event(enable_timing=True)
        evb.record(stream)
        bvh = BVH(gs)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        acc = path_trace(bvh, gs, cam, params, 0, params.spp, counters=counters, ws=ws)
        ev1.record(stream)
        img = resolve(acc, params.spp)
        return img, (ev0, ev1, evb)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        _log(f"warmup step {i} done")
    torch.cuda.synchronize()
    counters.zero_()
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        img, ev = step()
        evs.append(ev)
        if args.steps > 1:
            _log(f"step {i} issued")
    torch.cuda.synchronize()
    _log("timed steps done")
    wall = time.perf_counter() - t0
    c = counters.cpu().numpy().astype(np.float64)
    segments, paths, rounds, tests, blended, visits = (c[i] / args.steps for i in range(6))
    pt_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in evs]))
    build_ms = float(np.mean([c.elapsed_time(a) for a, b, c in evs]))
    ms_per_step = wall / args.steps * 1e3
    value = segments / (ms_per_step * 1e-3) / 1e6
    algo_bytes = blended * ALGO_BYTES_PER_HIT + segments * ALGO_BYTES_PER_SEGMENT
    achieved = algo_bytes / (pt_ms * 1e-3) / 1e9
    rec = {
        "metric": "Mrays/s multi-bounce PT over 2D Gaussians",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"path tracing, {scene.n} surfels in an 8x6x3 m room with 40 boxes, "
                               f"{cam.width}x{cam.height}, {params.spp} spp, max depth {params.max_depth}, "
                               f"RR from {params.rr_start}, k-buffer 16; step = BVH build + path tracing + resolve",
                   "surfels": scene.n, "width": cam.width, "height": cam.height, "spp": params.spp,
                   "max_depth": params.max_depth},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 5),
                     "traffic": measured_traffic() if args.spp is None and args.surfels is None else None},
        "detail": {"segments_per_step": segments, "paths_per_step": paths, "kbuf_rounds_per_segment":
                   round(rounds / max(segments, 1), 3), "candidate_tests_per_segment": round(tests / max(segments, 1), 2),
                   "nodes_visited_per_segment": round(visits / max(segments, 1), 2),
                   "blended_hits_per_segment": round(blended / max(segments, 1), 3),
                   "pt_kernel_ms": round(pt_ms, 3), "bvh_build_ms": round(build_ms, 3), "paths_per_s": round(paths / (ms_per_step * 1e-3), 1),
                   "image_mean": float(img.mean())},
    }
    if not args.no_cpu:
        _log("oracle CPU baseline")
        rec["cpu_baseline"] = cpu_baseline(scene, cam, params, segments)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
