#!/usr/bin/env python3
"""Benchmark of the occlusion-point-reuse hot path on one MI355X.

Workload (default): ambient occlusion at 1920x1080 over a displaced terrain
(512x512 cells, fBm heights) with 2000 level-2 icospheres (1,164,288
triangles), 1 sample per pixel, AO radius 2 m, 7x7 reuse window; synthetic,
seeded inputs standing in for the paper's scenes.

One step = the whole per-frame path on one batch of input (a new sample
index each step): occluder tracing (sample generation fused), the no-reuse
estimate, the biased 7x7 reuse, the first-hit validation rays and the
unbiased 7x7 reuse.  `value` is Mrays/s over the whole step: traced primary
rays per second.  Inputs are resident in HBM before the timed region.

Per-kernel times come from HIP events on the stream the library launches
on (torch's current stream, passed through the C-ABI).  The roofline entry
is for the kernel with the largest share of the step.  The CPU baseline is
the oracle on a bounded sample of the same frame.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 VALU rate with packed FP32 disabled, one op per lane per cycle:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T ops/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# FP32 operations of one test of one segment, counted from the kernels:
# box: 6 subtractions + 6 multiplies (slabs), 6 min/max (per-axis order),
# 3 max + 2 min (entry/exit), 1 scale, 1 clamp, 1 compare = 26;
# watertight triangle: 9 translations, 18 (shear), 9 (edge functions),
# 6 (sign tests), 2 (determinant), 9 (depths), 3 (T), 1 division, 2 compares = 59
OPS_BOX, OPS_TRI = 26, 59

WORKLOADS = {
    "ao_1080p": dict(mode="ao", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2, sample_seed=1),
    "shadow_1080p": dict(mode="shadow", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2,
                         sample_seed=1),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ao_1080p", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-baseline", default="on", choices=["on", "off"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-oracle work for the baseline")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (a frame would shard by image "
              "bands with halo recompute, see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2607_23122_amd as ocr
    import workloads as w

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    cfg = WORKLOADS[args.workload]
    mode, W, H, R, r = cfg["mode"], cfg["width"], cfg["height"], cfg["radius"], cfg["window_r"]
    t0 = time.time()
    scene = w.terrain_scene(cfg["scene_seed"])
    gb = w.render_gbuffer(scene, w.terrain_camera(W, H))
    light = w.terrain_light() if mode == "shadow" else None
    log(f"[bench] inputs {time.time() - t0:.1f}s: {scene.ntris} tris, {W}x{H}, valid {gb.valid.mean():.3f}")

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    bvh = ocr.build_bvh(scene.V, scene.F)
    info = bvh.info()
    dg = ocr.DeviceGBuffer.from_host(gb, dev)
    occ = ocr.Occluders.empty(H, W, dev)
    p_none = ocr.reuse_params("window", r, 0, "none")
    p_b = ocr.reuse_params("window", r, 0, "biased")
    p_u = ocr.reuse_params("window", r, 0, "unbiased", validated=True)
    ws = torch.empty(ocr.workspace_bytes(W, H, p_u), dtype=torch.uint8, device=dev)
    out_n = torch.empty((H, W), dtype=torch.float32, device=dev)
    out_b = torch.empty((H, W), dtype=torch.float32, device=dev)
    out_u = torch.empty((H, W), dtype=torch.float32, device=dev)
    _, _, kind = ocr.sample_rays(dg, mode, light, cfg["sample_seed"], 0)
    rays = int((kind == 0).sum().item())
    torch.cuda.synchronize()
    log(f"[bench] bvh {info.nnodes} nodes depth {info.depth} built in {info.build_ms:.0f} ms; {rays} traced rays/step")

    names = ["trace", "noreuse", "reuse_biased", "validate", "reuse_unbiased"]

    def step(s, ev=None):
        def mark(k):
            if ev is not None:
                ev[k].record(stream)
        mark(0)
        ocr.trace_occluders(bvh, dg, mode, R, light, cfg["sample_seed"], s, occ)
        mark(1)
        if mode == "ao":
            ocr.reuse_ao(None, dg, occ, R, p_none, out_n)
            mark(2)
            ocr.reuse_ao(None, dg, occ, R, p_b, out_b)
            mark(3)
            ocr.validate_pairs(bvh, dg, occ, mode, R, None, p_u, ws)
            mark(4)
            ocr.reuse_ao(None, dg, occ, R, p_u, out_u, ws)
        else:
            ocr.reuse_shadow(None, dg, occ, light, p_none, out_n)
            mark(2)
            ocr.reuse_shadow(None, dg, occ, light, p_b, out_b)
            mark(3)
            ocr.validate_pairs(bvh, dg, occ, mode, R, light, p_u, ws)
            mark(4)
            ocr.reuse_shadow(None, dg, occ, light, p_u, out_u, ws)
        mark(5)

    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * 2 ** 20 // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for s in range(args.warmup):
        step(1000 + s)
    torch.cuda.synchronize()

    # timed region: K steps with per-kernel events
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for s in range(args.steps):
        step(s, events[s])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    ms_per_step = total_ms / args.steps
    per = {n: float(np.mean([events[s][k].elapsed_time(events[s][k + 1]) for s in range(args.steps)]))
           for k, n in enumerate(names)}
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f}); " +
        ", ".join(f"{k} {v:.3f}" for k, v in per.items()))

    # work counted by the validation walk for one sample (outside the timed region)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    ocr.trace_occluders(bvh, dg, mode, R, light, cfg["sample_seed"], args.steps - 1, occ)
    ocr.validate_pairs(bvh, dg, occ, mode, R, light, p_u, ws, stats=stats)
    torch.cuda.synchronize()
    walks, nodes, box_tests, tri_tests = [int(v) for v in stats.cpu().tolist()]
    valid_px = int(gb.valid.sum())
    hits = int((occ.hit_u32() < ocr.HIT_SELF).sum())
    # Algorithmic bytes of one reuse launch: the G-buffer (pos, nrm, prim:
    # 28 B/px), the records (dz, nz, hit: 28 B/px) and the output (4 B/px).
    reuse_bytes = 60.0 * W * H
    reuse_gbs = reuse_bytes / (per["reuse_biased"] * 1e-3) / 1e9
    # pair densities a window launch evaluates: (4r+1)^2 per candidate
    pair_evals = hits * (4 * r + 1) ** 2
    dominant = max(names, key=lambda n: per[n])
    val_tops = (OPS_BOX * box_tests + OPS_TRI * tri_tests) / (per["validate"] * 1e-3) / 1e12
    if dominant == "validate":
        # traversal is VALU-bound: price the useful box and triangle tests
        roof = dict(bound="alu", achieved=round(val_tops, 3), peak=round(VALU_PEAK_TOPS, 1), unit="TFLOP/s",
                    frac=round(val_tops / VALU_PEAK_TOPS, 4), traffic=None, kernel="validate_window_kernel")
    else:
        roof = dict(bound="hbm", achieved=round(reuse_gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(reuse_gbs / HBM_PEAK_GBS, 5), traffic=None, kernel=dominant)

    result = {
        "metric": "Mrays/s + reuse-pass GB/s at 1080p; frames/s and p99 frame latency served",
        "value": round(rays / (ms_per_step * 1e-3) / 1e6, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: terrain 512x512 cells + 2000 icospheres ({scene.ntris} tris), "
                               f"{W}x{H}, 1 spp, R={R} m, 7x7 window, no-reuse + biased + unbiased",
                   "global_batch": 1, "seq_len": W * H, "parallelism": "single-gpu"},
        "kernels_ms": {k: round(v, 4) for k, v in per.items()},
        "trace_mrays_s": round(rays / (per["trace"] * 1e-3) / 1e6, 1),
        "reuse_gbs": round(reuse_gbs, 1),
        "reused_samples_per_s": round(hits * (2 * r + 1) ** 2 / (per["reuse_biased"] * 1e-3), 1),
        "pair_densities_per_s": round(pair_evals / (per["reuse_biased"] * 1e-3), 1),
        "biased_frame_ms": round(per["trace"] + per["reuse_biased"], 4),
        "rays_per_step": rays,
        "occluder_hits": hits,
        "valid_pixels": valid_px,
        "validation": {"walks": walks, "node_visits": nodes, "box_tests": box_tests, "tri_tests": tri_tests,
                       "segments_per_s": None, "useful_tflops": round(val_tops, 3)},
        "bvh": {"nodes": info.nnodes, "depth": info.depth, "device_mb": round(info.device_bytes / 2 ** 20, 1),
                "build_ms": round(info.build_ms, 1)},
        "roofline": roof,
    }

    if args.cpu_baseline == "on":
        result["cpu_baseline"] = cpu_baseline(scene, gb, cfg, light, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def cpu_baseline(scene, gb, cfg, light, budget_s):
    """The oracle, as it stands, on 64x64-target tiles of the same frame:
    records for each tile's halo, then the no-reuse, biased and unbiased
    estimates, until about budget_s seconds of work; Mrays/s = target pixels
    completed per second."""
    import numpy as np

    import oracle
    sc = oracle.Scene(scene.V, scene.F)
    W, H, r = gb.width, gb.height, cfg["window_r"]
    mode, R = cfg["mode"], cfg["radius"]
    rng = np.random.default_rng(7)
    done_px, ntiles = 0, 0
    t0 = time.perf_counter()
    while True:
        x = int(rng.integers(0, W - 64))
        y = int(rng.integers(0, H - 64))
        t = (x, y, x + 64, y + 64)
        for est in ("none", "biased", "unbiased"):
            p = oracle.params(mode, est, "window", radius=r, ao_radius=R, light=light, seed=cfg["sample_seed"])
            rec = oracle.records(sc, gb, p, oracle.halo_region(p, W, H, t))
            oracle.reuse(sc, gb, p, rec, t)
        done_px += 64 * 64
        ntiles += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": round(done_px / el / 1e6, 4), "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{ntiles} random 64x64-pixel tiles of the same frame (with their 3-pixel halos), "
                      f"records + no-reuse + biased + unbiased 7x7, {el:.1f} s on {cpu_model()}"}


if __name__ == "__main__":
    main()
