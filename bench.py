"""Benchmark: multi-bounce path tracing over 2D Gaussian surfels on one GPU.

Workload (one step): a 1M-surfel 8x6x3 m room with 40 furniture boxes and
~0.5% emissive ceiling-panel surfels (scene seed 3), one 1024x768 camera at
(1.0, 3.0, 1.6) looking at (8.0, 3.0, 1.2), 64 spp, max depth 5, Russian
roulette from depth 3, 16-entry k-buffer. A step is the whole hot path on
resident inputs: LBVH build over the surfels, the persistent path-tracing
kernel over all 50.3M paths, and the resolve of the fixed-point image.

Metric: ray segments traced per second (Mrays/s), counted on the device.
The roofline entry prices the path-tracing kernel by its algorithmic bytes:
68 B per blended hit (the canonical surfel record: centre, quaternion,
scales, opacity, albedo, radiance, emissive) plus 96 B of path state per
segment, over the kernel's duration from HIP events on its stream.

The CPU baseline times the FP64 brute-force oracle on a fixed sample of the
same workload's paths on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0
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


def cpu_baseline(scene, cam, params, budget_paths=96):
    """Oracle segments/s on a fixed sample of the workload's paths, across
    the host cores with a fork pool."""
    import multiprocessing as mp

    from oracle import Params
    from oracle.tracer import Scene64
    prm = Params(spp=params.spp, max_depth=params.max_depth, rr_start=params.rr_start, seed=params.seed,
                 camera_id=params.camera_id)
    _ORACLE.update(sc=Scene64(scene), cam=cam, prm=prm)
    rng = np.random.default_rng(7)
    pix = rng.choice(cam.width * cam.height, budget_paths, replace=False)
    samp = rng.integers(0, params.spp, budget_paths)
    cores = min(os.cpu_count() or 1, 16, budget_paths)
    jobs = [(np.array([p]), [int(s)]) for p, s in zip(pix, samp)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    segs = sum(r[0] for r in res)
    return {"value": segs / wall / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"{budget_paths} random (pixel, sample) paths of the same frame, {segs} segments, "
                      f"{wall:.1f} s wall on {cores} processes"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--surfels", type=int, default=1_000_000)
    ap.add_argument("--spp", type=int, default=None, help="override the workload's 64 spp (diagnostics only)")
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

    import scenegen as sg
    from paper_2601_23065_amd.api import BVH, Params, Scene, path_trace, path_trace_workspace, resolve

    scene, cams, cfg = sg.config(3, n_override=args.surfels if args.surfels != 1_000_000 else None)
    cam = cams[0]
    params = Params(spp=args.spp or cfg["spp"], max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0,
                    camera_id=0)
    _log(f"scene ready: {scene.n} surfels, {cam.width}x{cam.height}, {params.spp} spp")
    gs = Scene(scene.arrays())
    ws = path_trace_workspace(gs)
    counters = torch.zeros(6, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        bvh = BVH(gs)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        acc = path_trace(bvh, gs, cam, params, 0, params.spp, counters=counters, ws=ws)
        ev1.record(stream)
        img = resolve(acc, params.spp)
        return img, (ev0, ev1)

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
    pt_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
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
                               f"RR from {params.rr_start}, k-buffer 16; step = LBVH build + path tracing + resolve",
                   "surfels": scene.n, "width": cam.width, "height": cam.height, "spp": params.spp,
                   "max_depth": params.max_depth},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": None},
        "detail": {"segments_per_step": segments, "paths_per_step": paths, "kbuf_rounds_per_segment":
                   round(rounds / max(segments, 1), 3), "candidate_tests_per_segment": round(tests / max(segments, 1), 2),
                   "nodes_visited_per_segment": round(visits / max(segments, 1), 2),
                   "blended_hits_per_segment": round(blended / max(segments, 1), 3),
                   "pt_kernel_ms": round(pt_ms, 3), "paths_per_s": round(paths / (ms_per_step * 1e-3), 1),
                   "image_mean": float(img.mean())},
    }
    if not args.no_cpu:
        _log("oracle CPU baseline")
        rec["cpu_baseline"] = cpu_baseline(scene, cam, params)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
