#!/usr/bin/env python3
"""Benchmark of the occlusion-point-reuse hot path on one MI355X.

Workload ao_1080p (default): ambient occlusion at 1920x1080 over a displaced
terrain (512x512 cells, fBm heights) with 2000 level-2 icospheres (1,164,288
triangles), 1 sample per pixel, AO radius 2 m, 7x7 reuse window; synthetic,
seeded inputs standing in for the paper's scenes.  shadow_1080p: the same
with the 1 x 1 m rectangular light; shadow_sa_1080p and di_1080p: its shadows
under the solid-angle definition and its direct illumination;
shadow_sa_bilinear_1080p: solid-angle shadows with the light sampled from the
bilinear (general, receiver-dependent) emitter density; shadow2_1080p:
shadows of two lights.

One step = the whole per-frame path on one batch of input (a new sample
index each step): occluder tracing (sample generation fused), the no-reuse
estimate, the biased 7x7 reuse, the first-hit validation rays and the
unbiased 7x7 reuse.  `value` is Mrays/s over the whole step: traced primary
rays per second.  Inputs are resident in HBM before the timed region.

batched_16: sixteen views of uneven size (640x360 .. 2560x1440, 24,652,800
px) over four terrain scenes (50k .. 2M triangles), AO on even views and
shadows on odd ones, biased 7x7, as one autotuned plan (persistent trace and
reuse launches replayed from a HIP graph); a step is one plan launch, the
baseline sixteen separate per-view launch pairs.

served: Poisson arrivals over eight resident scenes and a pool of 720p,
1080p and 1440p G-buffers per scene, AO or shadow at 1 spp with biased 7x7
reuse, admitted under an HBM budget onto 8 stream slots; the baseline is a
one-slot FIFO server on the same arrival trace.

Per-kernel times come from HIP events on the stream the library launches
on (torch's current stream, passed through the C-ABI).  The roofline entry
is for the kernel with the largest share of the step.  The CPU baseline is
the oracle on a bounded sample of the same work.
"""
import argparse
import json
import os
import platform
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 VALU peak with packed FP32 disabled (the build turns it off): one
# instruction per lane per cycle, an FMA counting as two operations, as in the
# op counts below (a slab plane's subtract and multiply are one FMA):
# 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz = 78.6 TFLOP/s.  (The published
# 157.3 TFLOP/s needs packed FP32.)  Ops that are not FMAs (min/max, compares,
# selects) count once but take a full issue slot, so an op mix like the box
# test's (12 of its 26 ops in 6 FMAs; 17 instructions with three-operand
# min/max) tops out near 26 / 34 = 0.76 of this peak.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# MI355X's published FP32 vector peak (packed FP32 issue): the roofline's
# `peak`; the unpacked rate above is reported beside it
PUBLISHED_FP32_TOPS = 157.3


def alu_roof(tops, **extra):
    """An ALU roofline entry: achieved useful TFLOP/s against the published
    FP32 peak, and against the unpacked issue rate the build can reach."""
    d = dict(bound="alu", achieved=round(tops, 3), peak=PUBLISHED_FP32_TOPS, unit="TFLOP/s",
             frac=round(tops / PUBLISHED_FP32_TOPS, 4), peak_unpacked=round(VALU_PEAK_TOPS, 1),
             frac_unpacked=round(tops / VALU_PEAK_TOPS, 4))
    d.update(extra)
    return d
# FP32 operations of one test of one ray or segment, counted from the kernels
# (the counted tests are those each ray or segment needs on its own; lanes
# of a wave that execute a test their segment does not need are not useful
# work):
# box: 6 subtractions + 6 multiplies (slabs), 6 min/max (per-axis order),
# 3 max + 2 min (entry/exit), 1 scale, 1 clamp, 1 compare = 26;
# watertight triangle: 9 translations, 18 (shear), 9 (edge functions),
# 6 (sign tests), 2 (determinant), 9 (depths), 3 (T), 1 division, 2 compares = 59
OPS_BOX, OPS_TRI = 26, 59
# FP32 operations of one pair density, counted from the kernels: the pair
# vector w = (o_j - o_k) + dz_j (6), then AO: three dot products (9), three
# support compares, |w|^4 (1), a reciprocal and two products, a select = 17;
# shadow: five dot products (15), a reciprocal, s, two FMAs (a, b), six
# support compares and two abs, s^2 and the Jacobian ratio (3), a select = 31.
OPS_DENS = {"ao": 6 + 17, "shadow": 6 + 31}
OPS_DENS["shadow_sa"] = OPS_DENS["shadow"]
# solid-angle shadows scatter p/P times g = cos / |x - y'|^2 per (target,
# candidate) pair: the pair vector (6), two dot products (10), two
# reciprocals, a reciprocal square root, s, s^2 |w|^2 (2) and three products = 24
OPS_SA_G = 24
# direct illumination adds the receiver cosine: a dot product, a reciprocal
# square root and two products
OPS_DI_G = OPS_SA_G + 8
OPS_DENS["di"] = OPS_DENS["shadow"]
OPS_DENS["shadow2"] = 2 * OPS_DENS["shadow"]  # the density summed over two lights
# the bilinear emitter density: q(a, b) per pair density (three FMAs and a
# product = 7) and 1 / q(y') per scattered term (three dot products (15), two
# reciprocals, s, two FMAs (a, b), three FMAs for q and a product = 29)
OPS_BILIN_DENS, OPS_BILIN_G = 7, 29


def window_reuse_ops(r, mode, bilinear=False):
    """Useful FP32 ops per hit candidate of a window-r reuse launch: the
    (4r+1)^2 pair densities, the (4r+1)(2r+1) row box sums and (2r+1)^2
    column box sums of 2r adds each, and a reciprocal and product per target."""
    side, tw = 4 * r + 1, 2 * r + 1
    g = tw * tw * {"shadow_sa": OPS_SA_G, "di": OPS_DI_G}.get(mode, 0)
    if bilinear:
        g += side * side * OPS_BILIN_DENS + tw * tw * OPS_BILIN_G
    return side * side * OPS_DENS[mode] + side * tw * 2 * r + tw * tw * 2 * r + tw * tw * 2 + g

WORKLOADS = {
    "ao_1080p": dict(mode="ao", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2, sample_seed=1),
    "shadow_1080p": dict(mode="shadow", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2,
                         sample_seed=1),
    # shadows under the solid-angle definition: same records and validation
    "shadow_sa_1080p": dict(mode="shadow_sa", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2,
                            sample_seed=1),
    # occluder-domain direct illumination (Lambertian receivers, albedo 0.8,
    # the light at radiance 100): same records and validation
    # shadows of two rectangular lights (the 1 m light and a tilted 2 m x 1 m one)
    "shadow2_1080p": dict(mode="shadow2", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2,
                          sample_seed=1),
    "di_1080p": dict(mode="di", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2, sample_seed=1),
    # solid-angle shadows with the light sampled from the bilinear (general,
    # receiver-dependent) emitter density
    "shadow_sa_bilinear_1080p": dict(mode="shadow_sa", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2,
                                     sample_seed=1, light_pdf=1),
    "batched_16": dict(radius=2.0, window_r=3, sample_seed=1),
    # GROUP N = 8 reuse alone on the 1080p frame (the HBM-bound reuse variant)
    "group8_1080p": dict(mode="ao", width=1920, height=1080, radius=2.0, window_r=3, scene_seed=2, sample_seed=1),
    "served": dict(radius=2.0, window_r=3, rate=400.0, budget_gib=4.0, slots=8),
}
# served scenes: the batched generator's sizes twice, seeds 100..107
SERVED_SCENES = [dict(seed=100 + i, cells=c, spheres=n)
                 for i, (c, n) in enumerate([(128, 54), (256, 375), (512, 2000), (768, 2560)] * 2)]
SERVED_SIZES = [(1280, 720), (1920, 1080), (2560, 1440)]


TRACE_TU = ["density.hpp", "lights.hpp", "ocr_common.hpp", "trace.hip", "trace_pixel.hpp", "traverse.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ao_1080p_hbm_traffic.md")


def measured_traffic(kernel):
    """Calibrated HBM bytes (read + write) per launch of `kernel` from the
    committed counter summary, or None when the kernel's sources changed
    since the counters were taken (or no summary covers it)."""
    import hashlib
    try:
        txt = open(TRAFFIC_FILE).read()
        h = hashlib.sha256()
        for f in TRACE_TU:
            with open(os.path.join(ROOT, "paper_2607_23122_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        rec = txt.split("source_sha256:")[1].split()[0]
        table = json.loads(txt.split("traffic_json:")[1].strip().splitlines()[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec != h.hexdigest() or kernel not in table:
        return None
    return int(table[kernel]["read_bytes"] + table[kernel]["write_bytes"])


def alu_roofline(stats, ms, kernel):
    """Useful FP32 ops of the counted box and triangle tests per launch over
    the launch's average duration, against the VALU peak."""
    ops = OPS_BOX * stats[2] + OPS_TRI * stats[3]
    tops = ops / (ms * 1e-3) / 1e12
    return alu_roof(tops, traffic=None, kernel=kernel,
                    work={"walks": int(stats[0]), "node_visits": int(stats[1]), "box_tests": int(stats[2]),
                          "tri_tests": int(stats[3])})


def counted_trace(ocr, torch, bvh, dg, mode, R, light, seed, sample):
    stats = torch.zeros(5, dtype=torch.int64, device="cuda")
    ocr.trace_occluders_counted(bvh, dg, stats, mode, R, light, seed, sample)
    torch.cuda.synchronize()
    return [int(v) for v in stats.cpu().tolist()]


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
    ap.add_argument("--settle-seconds", type=float, default=1.0,
                    help="untimed steps before the warm-up until this much wall time has passed (clocks settle)")
    ap.add_argument("--workload", default="ao_1080p", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-baseline", default="on", choices=["on", "off"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-oracle work for the baseline")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size (to scale HBM byte counters)")
    ap.add_argument("--served-seconds", type=float, default=10.0, help="measured arrival window (served)")
    ap.add_argument("--served-warmup-seconds", type=float, default=2.0, help="arrivals before measuring (served)")
    ap.add_argument("--served-poses", type=int, default=2, help="camera poses per scene and resolution (served)")
    ap.add_argument("--served-baseline", default="on", choices=["on", "off"],
                    help="also run the one-slot FIFO server on the same arrivals")
    ap.add_argument("--served-rates", type=lambda v: [float(x) for x in v.split(",") if x], default=None,
                    help="further offered loads (requests/s), served and FIFO on the same arrivals; default: "
                         "midway between the two servers' measured capacities")
    ap.add_argument("--amortised-reps", type=int, default=3,
                    help="repetitions of 200 accumulated samples for the amortised per-sample times (0: off)")
    ap.add_argument("--extras", default="on", choices=["on", "off"],
                    help="with the default workload, also measure the shadow frame, GROUP 8 reuse, the batched "
                         "plan and the served loop, each as an object of the same JSON line")
    ap.add_argument("--primer", default="off", choices=["on", "off"],
                    help="first run a short AO frame step in a child process (a slow first GPU process was "
                         "once seen on freshly started machines; not seen since the trace kernel lost its "
                         "private stack)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (a frame would shard by image "
              "bands with halo recompute); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    # (counting devices does not initialise the GPU in this process)
    if torch.cuda.device_count() == 0:
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    primer = run_primer() if args.primer == "on" else None
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched_16":
        result = run_batched(args)
    elif args.workload == "served":
        result = run_served(args)
    elif args.workload == "group8_1080p":
        g8 = run_group8(args, {})
        result = {"metric": "GROUP 8 reuse GB/s of algorithmic bytes at 1080p (AO and shadows)",
                  "value": g8["ao"]["biased_gbs"], "unit": "GB/s", "n_gpus": 1, "steps": 30, "warmup": 5,
                  "ms_per_step": g8["ao"]["biased_ms"], "higher_is_better": True, "scaling": "weak",
                  "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                  "config": {"workload": "group8_1080p: the 1080p terrain frame, GROUP N = 8 (4x2 groups), biased "
                                         "and unbiased, and no reuse", "global_batch": 1, "seq_len": 1920 * 1080,
                             "parallelism": "single-gpu"},
                  "group8_reuse": g8,
                  "roofline": {"bound": "hbm", "achieved": g8["ao"]["biased_gbs"], "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": g8["ao"]["biased_hbm_frac"], "traffic": None,
                               "kernel": "ocr::reuse_group_kernel<0, false, ocr::LightF, 4, 2>"}}
    elif args.workload == "ao_1080p" and args.extras == "on":
        result = run_all(args)
    else:
        result = run_frame(args, amortised_reps=args.amortised_reps)
    result["primer"] = primer
    print(json.dumps(result), flush=True)


def run_primer():
    """Runs a short AO frame step (two steps after a second of settle steps)
    in a child process before this process touches the GPU, and returns the
    child's trace time (--primer on).  On freshly started machines the first
    process that used the GPU was once seen to run the trace kernel about 13x
    slower for its whole life, while the trace kernel used private memory;
    the child takes that place.  A failing child ends the bench with its
    status: the GPU is not used again after a failure."""
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "ao_1080p", "--steps", "2", "--warmup", "0",
           "--settle-seconds", "1.0", "--cpu-baseline", "off", "--primer", "off", "--extras", "off",
           "--amortised-reps", "0"]
    t0 = time.perf_counter()
    try:
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    except subprocess.TimeoutExpired:
        log("[bench] primer process timed out")
        sys.exit(124)
    if p.returncode != 0:
        log(p.stderr[-4000:])
        log(f"[bench] primer process failed with status {p.returncode}")
        sys.exit(p.returncode if p.returncode > 0 else 1)
    m = re.findall(r"steps: .*?; trace ([0-9.]+)", p.stderr)
    trace_ms = float(m[-1]) if m else None
    log(f"[bench] primer process: {time.perf_counter() - t0:.1f} s, trace {trace_ms} ms/step")
    return {"seconds": round(time.perf_counter() - t0, 1), "trace_ms": trace_ms}


def settle(torch, fn, seconds, max_calls=2000):
    """Untimed repetitions of fn until `seconds` of wall time have passed (at
    most max_calls): a fresh GPU can run its first second of work at lower
    clocks, which the W warm-up steps alone do not always cover."""
    t0 = time.perf_counter()
    k = 0
    while k < max_calls and time.perf_counter() - t0 < seconds:
        fn(k)
        k += 1
        if k % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def frame_inputs(ctx, cfg):
    """The 1080p terrain scene, its G-buffer and BVH (built once, shared by
    the frame workloads of one run)."""
    import paper_2607_23122_amd as ocr
    import workloads as w
    key = (cfg["scene_seed"], cfg["width"], cfg["height"])
    if ctx.get("key") != key:
        t0 = time.time()
        scene = w.terrain_scene(cfg["scene_seed"])
        gb = w.render_gbuffer(scene, w.terrain_camera(cfg["width"], cfg["height"]))
        t_in = time.time() - t0
        bvh = ocr.build_bvh(scene.V, scene.F)
        ctx.clear()
        ctx.update(key=key, scene=scene, gb=gb, bvh=bvh, dg=ocr.DeviceGBuffer.from_host(gb, "cuda:0"), t_in=t_in)
    return ctx["scene"], ctx["gb"], ctx["bvh"], ctx["dg"]


def calibration_copy(torch, args):
    """One device-to-device copy of --calibration-copy-mib MiB (none at 0):
    a kernel of known traffic to scale the HBM byte counters by."""
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * 2 ** 20 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b


def run_frame(args, workload=None, ctx=None, cpu_seconds=None, amortised_reps=0):
    import numpy as np
    import torch

    import paper_2607_23122_amd as ocr
    import workloads as w

    workload = workload or args.workload
    ctx = {} if ctx is None else ctx
    cpu_seconds = args.cpu_seconds if cpu_seconds is None else cpu_seconds
    cfg = WORKLOADS[workload]
    mode, W, H, R, r = cfg["mode"], cfg["width"], cfg["height"], cfg["radius"], cfg["window_r"]
    scene, gb, bvh, dg = frame_inputs(ctx, cfg)
    light = w.terrain_light() if mode != "ao" else None
    if mode == "shadow2":
        light = w.two_lights()
    bilinear = cfg.get("light_pdf", 0) == 1
    if bilinear:
        light.pdf = 1
    tmode = "shadow" if mode in ("shadow_sa", "di", "shadow2") else mode  # the mode records are traced in
    log(f"[bench] {workload}: inputs {ctx['t_in']:.1f}s: {scene.ntris} tris, {W}x{H}, valid {gb.valid.mean():.3f}")

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    info = bvh.info()
    occ = ocr.Occluders.empty(H, W, dev)
    p_none = ocr.reuse_params("window", r, 0, "none")
    p_b = ocr.reuse_params("window", r, 0, "biased")
    p_u = ocr.reuse_params("window", r, 0, "unbiased", validated=True)
    ws = torch.empty(ocr.workspace_bytes(W, H, p_u), dtype=torch.uint8, device=dev)
    out_n = torch.empty((H, W), dtype=torch.float32, device=dev)
    out_b = torch.empty((H, W), dtype=torch.float32, device=dev)
    out_u = torch.empty((H, W), dtype=torch.float32, device=dev)
    if mode == "shadow2":
        # (the sampler entry point takes one light: count the traced samples of a trace)
        ocr.trace_occluders(bvh, dg, tmode, R, light, cfg["sample_seed"], 0, occ)
        rays = int(((occ.hit_u32() != ocr.HIT_SELF) & gb.valid).sum())
    else:
        _, _, kind = ocr.sample_rays(dg, tmode, light, cfg["sample_seed"], 0)
        rays = int((kind == 0).sum().item())
    torch.cuda.synchronize()
    log(f"[bench] bvh {info.nnodes} nodes depth {info.depth} built in {info.build_ms:.0f} ms; {rays} traced rays/step")

    names = ["trace", "noreuse", "reuse_biased", "validate", "reuse_unbiased"]

    def step(s, ev=None):
        def mark(k):
            if ev is not None:
                ev[k].record(stream)
        mark(0)
        ocr.trace_occluders(bvh, dg, tmode, R, light, cfg["sample_seed"], s, occ)
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
            if mode == "di":
                def reuse(b, d, o, lt, p, out, ws=None):
                    return ocr.reuse_direct_illumination(b, d, o, lt, p, radiance=100.0, albedo=0.8, out=out,
                                                         workspace=ws)
            else:
                reuse = ocr.reuse_shadow_solid_angle if mode == "shadow_sa" else ocr.reuse_shadow
            reuse(None, dg, occ, light, p_none, out_n)
            mark(2)
            reuse(None, dg, occ, light, p_b, out_b)
            mark(3)
            ocr.validate_pairs(bvh, dg, occ, tmode, R, light, p_u, ws)
            mark(4)
            reuse(None, dg, occ, light, p_u, out_u, ws)
        mark(5)

    calibration_copy(torch, args)

    settle(torch, lambda k: step(2000 + k), args.settle_seconds)
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
    samples = {n: np.array([events[s][k].elapsed_time(events[s][k + 1]) for s in range(args.steps)])
               for k, n in enumerate(names)}
    per = {n: float(v.mean()) for n, v in samples.items()}
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f}); " +
        ", ".join(f"{k} {v:.3f}" for k, v in per.items()))

    # work counted by the validation walk for one sample (outside the timed region)
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    ocr.trace_occluders(bvh, dg, tmode, R, light, cfg["sample_seed"], args.steps - 1, occ)
    ocr.validate_pairs(bvh, dg, occ, tmode, R, light, p_u, ws, stats=stats)
    torch.cuda.synchronize()
    walks, nodes, box_tests, tri_tests, segments = [int(v) for v in stats.cpu().tolist()]
    valid_px = int(gb.valid.sum())
    # reported statistics: the fraction of valid pixels whose raw estimate is
    # negative (outputs are not clamped, and a sum of reuse weights can exceed
    # the unoccluded value)
    vmask = torch.from_numpy(gb.valid).to(dev)
    negative = {k: round(float((o[vmask] < 0).float().mean().item()), 6)
                for k, o in (("biased", out_b), ("unbiased", out_u))}
    hits = int((occ.hit_u32() < ocr.HIT_SELF).sum())
    # Algorithmic bytes of one reuse launch: the G-buffer (pos, nrm, prim:
    # 28 B/px), the records (dz, nz, hit: 28 B/px) and the output (4 B/px).
    reuse_bytes = 60.0 * W * H
    reuse_gbs = reuse_bytes / (per["reuse_biased"] * 1e-3) / 1e9
    # pair densities a window launch evaluates: (4r+1)^2 per candidate
    pair_evals = hits * (4 * r + 1) ** 2
    dominant = max(names, key=lambda n: per[n])
    # validation: the useful box and triangle tests of the segments plus the
    # pair densities deciding which pairs get a segment ((4r+1)^2 - 1 per candidate)
    val_ops = OPS_BOX * box_tests + OPS_TRI * tri_tests + hits * ((4 * r + 1) ** 2 - 1) * OPS_DENS[mode]
    val_tops = val_ops / (per["validate"] * 1e-3) / 1e12
    reuse_tops = hits * window_reuse_ops(r, mode, bilinear) / (per["reuse_biased"] * 1e-3) / 1e12
    if dominant == "validate":
        # traversal and densities are VALU-bound: price the useful operations
        # one validation per light type (single-light kernels carry LightF)
        lt = "ocr::LightSetF" if mode == "shadow2" else "ocr::LightF"
        kname = f"ocr::validate_window_kernel<{0 if mode == 'ao' else 1}, false, {lt}, false>"
        traffic = measured_traffic(kname) if workload == "ao_1080p" else None
        roof = alu_roof(val_tops, traffic=traffic, kernel=kname)
    elif dominant in ("reuse_biased", "reuse_unbiased"):
        # a 7x7 window reuse binds on the VALU (up to 169 densities per
        # candidate): its useful operations against the VALU peak, with its
        # algorithmic HBM rate beside them
        t_ms = per[dominant]
        tops = hits * window_reuse_ops(r, mode, bilinear) / (t_ms * 1e-3) / 1e12
        # (the unbiased launch also reads each pixel's validation words)
        vbytes = (((4 * r + 1) ** 2 + 31) // 32) * 4 * W * H if dominant == "reuse_unbiased" else 0
        gbs = (reuse_bytes + vbytes) / (t_ms * 1e-3) / 1e9
        lt = "ocr::LightSetF" if mode == "shadow2" else "ocr::LightBilinF" if bilinear else "ocr::LightF"
        kname = (f"ocr::reuse_window_kernel<{ {'ao': 0, 'shadow': 1, 'shadow_sa': 2, 'di': 3, 'shadow2': 1}[mode]}, "
                 f"{'true' if dominant == 'reuse_unbiased' else 'false'}, {lt}>")
        roof = alu_roof(tops, traffic=None, kernel=kname, hbm_gbs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
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
        "config": {"workload": f"{workload}: terrain 512x512 cells + 2000 icospheres ({scene.ntris} tris), "
                               f"{W}x{H}, 1 spp, R={R} m, 7x7 window, no-reuse + biased + unbiased"
                               + {"shadow2": ", shadows of two rectangular lights",
                                  "shadow_sa": ", shadows under the solid-angle definition",
                                  "di": ", occluder-domain direct illumination"}.get(mode, "")
                               + (", light sampled from the bilinear emitter density" if bilinear else ""),
                   "global_batch": 1, "seq_len": W * H, "parallelism": "single-gpu"},
        "kernels_ms": {k: round(v, 4) for k, v in per.items()},
        "kernels_ms_p50": {k: round(float(np.percentile(v, 50)), 4) for k, v in samples.items()},
        "kernels_ms_p90": {k: round(float(np.percentile(v, 90)), 4) for k, v in samples.items()},
        "trace_mrays_s": round(rays / (per["trace"] * 1e-3) / 1e6, 1),
        "reuse_gbs": round(reuse_gbs, 1),
        "reused_samples_per_s": round(hits * (2 * r + 1) ** 2 / (per["reuse_biased"] * 1e-3), 1),
        "pair_densities_per_s": round(pair_evals / (per["reuse_biased"] * 1e-3), 1),
        "biased_frame_ms": round(per["trace"] + per["reuse_biased"], 4),
        "reuse_roofline": alu_roof(reuse_tops, hbm_gbs=round(reuse_gbs, 1), hbm_frac=round(reuse_gbs / HBM_PEAK_GBS, 4),
                               kernel=f"ocr::reuse_window_kernel<{ {'ao': 0, 'shadow': 1, 'shadow_sa': 2, 'di': 3, 'shadow2': 1}[mode]}, false, "
                                      f"{'ocr::LightSetF' if mode == 'shadow2' else 'ocr::LightBilinF' if bilinear else 'ocr::LightF'}>",
                               ops_per_candidate=window_reuse_ops(r, mode, bilinear)),
        "rays_per_step": rays,
        "negative_pixel_fraction": negative,
        "occluder_hits": hits,
        "valid_pixels": valid_px,
        "validation": {"walks": walks, "node_visits": nodes, "box_tests": box_tests, "tri_tests": tri_tests,
                       "segments": segments,
                       "segments_per_s": round(segments / (per["validate"] * 1e-3), 1), "useful_tflops": round(val_tops, 3)},
        "bvh": {"nodes": info.nnodes, "depth": info.depth, "device_mb": round(info.device_bytes / 2 ** 20, 1),
                "build_ms": round(info.build_ms, 1)},
        "roofline": roof,
    }

    # (the counting trace takes one uniformly sampled light)
    result["trace_roofline"] = None if mode == "shadow2" or bilinear else alu_roofline(
        counted_trace(ocr, torch, bvh, dg, tmode, R, light, cfg["sample_seed"], args.steps - 1), per["trace"],
        "trace_kernel")
    if workload == "ao_1080p":
        result["trace_roofline"]["traffic"] = measured_traffic("ocr::trace_kernel<0, ocr::LightF>")
    if amortised_reps > 0 and mode in ("ao", "shadow"):
        result["amortised_ms_per_spp"] = amortised(ocr, torch, bvh, dg, occ, tmode, R, light, cfg["sample_seed"],
                                                   (p_none, p_b, p_u), ws, out_n, amortised_reps)
    if args.cpu_baseline == "on" and cpu_seconds > 0:
        # the GPU outputs of sample 0 (the oracle's tiles use the same sample)
        step(0)
        torch.cuda.synchronize()
        gpu = {"hit": occ.hit_u32(), "none": out_n.cpu().numpy(), "biased": out_b.cpu().numpy(),
               "unbiased": out_u.cpu().numpy()}
        result["cpu_baseline"], par = cpu_baseline(scene, gb, cfg, light, cpu_seconds, gpu)
        result["grazing_fraction"] = par["grazing_fraction"]
        result["excluded_fraction"] = par["excluded_fraction"]
        result["parity_sample"] = par
    return result


def amortised(ocr, torch, bvh, dg, occ, tmode, R, light, seed, params, ws, out, reps, spp=200):
    """The paper's amortised timing (the protocol of its absolute-runtime
    tables): each repetition accumulates `spp` samples of the whole per-sample
    pass into one buffer (trace, then the estimator: no reuse, biased, or
    validation + unbiased), the time of `reps` repetitions divided by the
    samples taken; ms per sample."""
    p_none, p_b, p_u = params
    stream = torch.cuda.current_stream()
    res = {}
    for name, p in (("noreuse", p_none), ("biased", p_b), ("unbiased", p_u)):
        def one_rep(base):
            for s in range(spp):
                ocr.trace_occluders(bvh, dg, tmode, R, light, seed, base + s, occ)
                acc = ocr.ReuseParams(p.pattern, p.radius, p.group_n, p.estimator, p.dark_guard, 0 if s == 0 else 1,
                                      p.validated)
                if p.estimator == 2:
                    ocr.validate_pairs(bvh, dg, occ, tmode, R, light, p, ws)
                if tmode == "ao":
                    ocr.reuse_ao(None, dg, occ, R, acc, out, ws)
                else:
                    ocr.reuse_shadow(None, dg, occ, light, acc, out, ws)
            ocr.scale(out, 1.0 / spp)
        one_rep(10_000)  # warm-up repetition
        torch.cuda.synchronize()
        ev = _events(torch, 2)
        ev[0].record(stream)
        for k in range(reps):
            one_rep(20_000 + k * spp)
        ev[1].record(stream)
        torch.cuda.synchronize()
        res[name] = round(ev[0].elapsed_time(ev[1]) / (reps * spp), 4)
    res["protocol"] = f"{spp} spp accumulated per repetition, {reps} repetitions, time / samples"
    log(f"[bench] amortised ms per sample: {res}")
    return res


FRAME_KEYS = ["value", "unit", "ms_per_step", "config", "kernels_ms", "kernels_ms_p50", "kernels_ms_p90",
              "trace_mrays_s", "reuse_gbs", "roofline", "reuse_roofline", "trace_roofline", "negative_pixel_fraction",
              "amortised_ms_per_spp", "grazing_fraction", "excluded_fraction", "parity_sample", "cpu_baseline"]


def run_all(args):
    """The default line: the 1080p AO step (the headline), then each further
    configuration's own headline as an object of the same line -- the 1080p
    shadow step, GROUP 8 reuse against the HBM roof, the batched plan and the
    served loop (shorter runs than their own workloads' defaults)."""
    import copy

    import torch
    ctx = {}
    t0 = time.time()
    result = run_frame(args, "ao_1080p", ctx, amortised_reps=args.amortised_reps)
    sh = run_frame(args, "shadow_1080p", ctx, cpu_seconds=min(4.0, args.cpu_seconds), amortised_reps=args.amortised_reps)
    result["shadow_1080p"] = {k: sh[k] for k in FRAME_KEYS if k in sh}
    result["group8_reuse"] = run_group8(args, ctx)
    ctx.clear()
    torch.cuda.empty_cache()
    log(f"[bench] frame workloads done at {time.time() - t0:.0f} s")
    a = copy.copy(args)
    a.cpu_baseline = "off"
    a.steps, a.warmup = min(args.steps, 10), min(args.warmup, 2)
    b = run_batched(a)
    result["batched_16"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "config", "mpx_per_s", "plan_ms",
                                              "plan_no_graph_ms", "per_view_pairs_ms", "speedup_vs_per_view",
                                              "tuning", "roofline")}
    torch.cuda.empty_cache()
    log(f"[bench] batched done at {time.time() - t0:.0f} s")
    a.served_seconds, a.served_warmup_seconds = min(args.served_seconds, 4.0), min(args.served_warmup_seconds, 1.0)
    a.served_poses = 1
    sv = run_served(a)
    result["served"] = {k: sv[k] for k in ("value", "unit", "config", "p50_ms", "p99_ms", "offered_gpx_per_s",
                                           "stable", "served", "fifo_one_slot", "capacity_frames_per_s",
                                           "higher_loads", "roofline")}
    log(f"[bench] served done at {time.time() - t0:.0f} s")
    return result


def run_group8(args, ctx, launches=30):
    """GROUP 8 reuse (the paper's own pattern: 4x2 pixel groups) and the
    no-reuse write-out on the 1080p frame, AO and shadows: median launch time
    over `launches` launches, and the algorithmic bytes' rate against the HBM
    roof.  Biased GROUP 8 reads the G-buffer (28 B/px) and the records
    (28 B/px) and writes the estimate (4 B/px); no reuse reads the G-buffer's
    primitive id and the hit id and writes the estimate (12 B/px)."""
    import numpy as np
    import torch

    import paper_2607_23122_amd as ocr
    import workloads as w

    cfg = WORKLOADS["ao_1080p"]
    W, H, R = cfg["width"], cfg["height"], cfg["radius"]
    scene, gb, bvh, dg = frame_inputs(ctx, cfg)
    calibration_copy(torch, args)
    stream = torch.cuda.current_stream()
    occ = ocr.Occluders.empty(H, W)
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    p_b = ocr.reuse_params("group", 0, 8, "biased")
    p_u = ocr.reuse_params("group", 0, 8, "unbiased", validated=True)
    p_n = ocr.reuse_params("group", 0, 8, "none")
    ws = torch.empty(ocr.workspace_bytes(W, H, p_u), dtype=torch.uint8, device="cuda")
    res = {}
    for mode in ("ao", "shadow"):
        light = w.terrain_light() if mode == "shadow" else None
        ocr.trace_occluders(bvh, dg, mode, R, light, cfg["sample_seed"], 0, occ)

        def reuse(p, wsp=None):
            if mode == "ao":
                ocr.reuse_ao(None, dg, occ, R, p, out, wsp)
            else:
                ocr.reuse_shadow(None, dg, occ, light, p, out, wsp)

        def timed(fn):
            for _ in range(5):
                fn()
            ev = _events(torch, 2 * launches)
            for k in range(launches):
                ev[2 * k].record(stream)
                fn()
                ev[2 * k + 1].record(stream)
            torch.cuda.synchronize()
            return float(np.median([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(launches)]))

        t_b = timed(lambda: reuse(p_b))
        t_v = timed(lambda: ocr.validate_pairs(bvh, dg, occ, mode, R, light, p_u, ws))
        t_u = timed(lambda: reuse(p_u, ws))
        t_n = timed(lambda: reuse(p_n))
        gbs_b = 60.0 * W * H / (t_b * 1e-3) / 1e9
        gbs_n = 12.0 * W * H / (t_n * 1e-3) / 1e9
        res[mode] = {"biased_ms": round(t_b, 4), "biased_gbs": round(gbs_b, 1),
                     "biased_hbm_frac": round(gbs_b / HBM_PEAK_GBS, 4),
                     "validate_ms": round(t_v, 4), "unbiased_reuse_ms": round(t_u, 4),
                     "noreuse_ms": round(t_n, 4), "noreuse_gbs": round(gbs_n, 1),
                     "noreuse_hbm_frac": round(gbs_n / HBM_PEAK_GBS, 4)}
    res["note"] = ("median event-timed launch; biased 60 B/px, no reuse 12 B/px of algorithmic bytes at "
                   f"{W}x{H}; HBM peak {HBM_PEAK_GBS:.0f} GB/s")
    log(f"[bench] group 8: {res}")
    return res


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def run_batched(args):
    import numpy as np
    import torch

    import paper_2607_23122_amd as ocr
    import workloads as w

    cfg = WORKLOADS["batched_16"]
    R, r, seed = cfg["radius"], cfg["window_r"], cfg["sample_seed"]
    t0 = time.time()
    scenes = [w.batch_scene(i) for i in range(4)]
    light = w.terrain_light()
    views = []
    for si, cam, mode in w.batch_views():
        views.append((si, w.render_gbuffer(scenes[si], cam), mode))
    px = sum(gb.width * gb.height for _, gb, _ in views)
    log(f"[bench] batched inputs {time.time() - t0:.1f}s: {[s.ntris for s in scenes]} tris, 16 views, {px} px")
    bvhs = [ocr.build_bvh(s.V, s.F) for s in scenes]
    dgs = [ocr.DeviceGBuffer.from_host(gb) for _, gb, _ in views]
    params = ocr.reuse_params("window", r, 0, "biased")
    outs = [torch.empty((gb.height, gb.width), dtype=torch.float32, device="cuda") for _, gb, _ in views]
    descs = [ocr.view_desc(bvhs[si], dgs[v], outs[v], mode, R, light if mode == "shadow" else None, seed, 0, params)
             for v, (si, gb, mode) in enumerate(views)]
    plan = ocr.Plan(descs)  # autotuned
    info = plan.info()
    tun = info.tuning
    log(f"[bench] autotuned: tile {tun.tile_w}x{tun.tile_h} packing {tun.packing}, trace {info.best_trace_ms:.3f} ms "
        f"({info.candidates} settings, {info.tune_ms:.0f} ms)")
    plan_eager = ocr.Plan(descs, ocr.PlanTuning(tun.tile_w, tun.tile_h, tun.packing, 0))
    stream = torch.cuda.current_stream()
    # per-view baseline: sixteen separate launch pairs into the same outputs
    occs = [ocr.Occluders.empty(gb.height, gb.width) for _, gb, _ in views]

    def per_view():
        for v, (si, gb, mode) in enumerate(views):
            lt = light if mode == "shadow" else None
            ocr.trace_occluders(bvhs[si], dgs[v], mode, R, lt, seed, 0, occs[v])
            if mode == "ao":
                ocr.reuse_ao(None, dgs[v], occs[v], R, params, outs[v])
            else:
                ocr.reuse_shadow(None, dgs[v], occs[v], light, params, outs[v])

    def timed(fn, steps, warm):
        settle(torch, lambda k: fn(), args.settle_seconds)
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        ev = _events(torch, 2)
        t = time.perf_counter()
        ev[0].record(stream)
        for _ in range(steps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps, (time.perf_counter() - t) * 1e3 / steps

    ms_plan, wall_plan = timed(plan.launch, args.steps, args.warmup)
    ms_eager, _ = timed(plan_eager.launch, args.steps, args.warmup)
    ms_pv, wall_pv = timed(per_view, args.steps, args.warmup)
    log(f"[bench] batched {ms_plan:.3f} ms/launch (wall {wall_plan:.3f}), no graph {ms_eager:.3f}, "
        f"16 per-view pairs {ms_pv:.3f} (wall {wall_pv:.3f})")
    # trace-phase time of the tuned plan, and the traced work (counted per view)
    plan_trace_ms = info.best_trace_ms
    work = np.zeros(5, np.int64)
    for v, (si, gb, mode) in enumerate(views):
        work += np.array(counted_trace(ocr, torch, bvhs[si], dgs[v], mode, R, light if mode == "shadow" else None,
                                       seed, 0), np.int64)
    frames_s = 16.0 / (ms_plan * 1e-3)
    result = {
        "metric": "frames/s, 16 batched views of uneven size (24.65 Mpx), biased 7x7",
        "value": round(frames_s, 1),
        "unit": "frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_plan, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_16: 4 terrain scenes " + str([s.ntris for s in scenes]) +
                               " tris, 16 orbit views 640x360..2560x1440, AO even / shadow odd, R=2 m, 7x7 biased, "
                               "one autotuned plan launch",
                   "global_batch": 16, "seq_len": px, "parallelism": "single-gpu"},
        "mpx_per_s": round(px / (ms_plan * 1e-3) / 1e6, 1),
        "plan_ms": round(ms_plan, 4),
        "plan_no_graph_ms": round(ms_eager, 4),
        "per_view_pairs_ms": round(ms_pv, 4),
        "speedup_vs_per_view": round(ms_pv / ms_plan, 3),
        "tuning": {"tile": f"{tun.tile_w}x{tun.tile_h}", "packing": ["row", "block8", "morton"][tun.packing],
                   "candidates": info.candidates, "tune_ms": round(info.tune_ms, 1),
                   "trace_phase_ms": round(plan_trace_ms, 4)},
        "roofline": alu_roofline(work, plan_trace_ms, "batch_trace_kernel"),
    }
    if args.cpu_baseline == "on":
        result["cpu_baseline"] = cpu_baseline_views(scenes, views, cfg, light, args.cpu_seconds, px / 16.0)
    return result


def run_served(args):
    import numpy as np
    import torch

    import paper_2607_23122_amd as ocr
    import workloads as w

    cfg = WORKLOADS["served"]
    R, r = cfg["radius"], cfg["window_r"]
    t0 = time.time()
    light = w.terrain_light()
    bvhs, pools, scenes = [], [], []
    for i, sc in enumerate(SERVED_SCENES):
        s = w.terrain_scene(seed=sc["seed"], cells=sc["cells"], nspheres=sc["spheres"])
        scenes.append(s)
        bvhs.append(ocr.build_bvh(s.V, s.F))
        pool = []
        for pose in range(args.served_poses):
            for (W, H) in SERVED_SIZES:
                cam = w.orbit_camera(pose * 3 + i, 8 * args.served_poses, W, H)
                pool.append(ocr.DeviceGBuffer.from_host(w.render_gbuffer(s, cam)))
        pools.append(pool)
        log(f"[bench] served scene {i}: {s.ntris} tris, {len(pool)} G-buffers ({time.time() - t0:.0f} s)")
    torch.cuda.synchronize()
    params = ocr.reuse_params("window", r, 0, "biased")
    rate = cfg["rate"]
    total_s = args.served_warmup_seconds + args.served_seconds
    px_of = [[dg.width * dg.height for dg in pool] for pool in pools]

    def trace_of(rate):
        """Poisson arrivals at `rate` over total_s (numpy seed 7), each
        picking (scene, G-buffer, AO or shadow) uniformly."""
        rng = np.random.default_rng(7)
        arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * total_s * 1.5) + 16))
        arr = arr[arr < total_s]
        pk = [(int(rng.integers(8)), int(rng.integers(len(pools[0]))), "ao" if rng.random() < 0.5 else "shadow")
              for _ in range(len(arr))]
        return arr, pk

    arrivals, picks = trace_of(rate)
    offered_gpx = sum(px_of[s][v] for s, v, _ in picks) / total_s / 1e9

    def serve(slots, arrivals=arrivals, picks=picks):
        srv = ocr.Server(int(cfg["budget_gib"] * 2 ** 30), slots=slots, poll_us=10)
        sids = [srv.add_scene(bvhs[i], pools[i]) for i in range(8)]
        start = ocr.server_now_ms() + 50.0
        lat = {}
        k = 0
        while len(lat) < len(arrivals):
            now = ocr.server_now_ms()
            while k < len(arrivals) and start + arrivals[k] * 1e3 <= now:
                si, vi, mode = picks[k]
                srv.submit(ocr.request(sids[si], vi, mode, R, light if mode == "shadow" else None, k, 0, params,
                                       None, start + arrivals[k] * 1e3))
                k += 1
            for res in srv.poll(1024):
                if res.status != 0:
                    raise RuntimeError(f"request failed: {res.status}")
                lat[res.ticket] = (res.arrival_ms - start, res.latency_ms, res.end_ms - start)
                srv.release(res.ticket)
            if k < len(arrivals):
                nxt = start + arrivals[k] * 1e3
                time.sleep(max(0.0, min(nxt - ocr.server_now_ms(), 1.0)) * 1e-3)
            else:
                time.sleep(0.0002)
        st = srv.stats()
        srv.destroy()
        warm = args.served_warmup_seconds * 1e3
        meas = [(a, l, e) for a, l, e in lat.values() if a >= warm]
        ls = np.sort(np.array([l for _, l, _ in meas]))
        span = (max(e for _, _, e in meas) - warm) * 1e-3

        def pct(q):
            return float(ls[min(len(ls) - 1, max(0, int(np.ceil(q * len(ls))) - 1))])
        return dict(requests=len(meas), offered_per_s=round(len(meas) / (args.served_seconds), 1),
                    frames_per_s=round(len(meas) / span, 1), p50_ms=round(pct(0.5), 3),
                    p99_ms=round(pct(0.99), 3), max_ms=round(float(ls[-1]), 3), mean_ms=round(float(ls.mean()), 3),
                    max_in_flight=int(st.max_in_flight), waited_for_memory=int(st.waited_for_memory),
                    peak_mb=round(st.peak_bytes / 2 ** 20, 1))

    def saturate(slots, n=1000):
        """Capacity: n requests of the same mix submitted at once (arrival =
        submission), completed frames/s from the first submission to the
        last completion."""
        srv = ocr.Server(int(cfg["budget_gib"] * 2 ** 30), slots=slots, poll_us=10)
        sids = [srv.add_scene(bvhs[i], pools[i]) for i in range(8)]
        t_first = ocr.server_now_ms()
        for k in range(n):
            si, vi, mode = picks[k % len(picks)]
            srv.submit(ocr.request(sids[si], vi, mode, R, light if mode == "shadow" else None, k, 0, params, None))
        done, last = 0, t_first
        while done < n:
            for res in srv.poll(1024):
                if res.status != 0:
                    raise RuntimeError(f"request failed: {res.status}")
                done += 1
                last = max(last, res.end_ms)
                srv.release(res.ticket)
            time.sleep(0.0002)
        srv.destroy()
        return round(n / ((last - t_first) * 1e-3), 1)

    log(f"[bench] served: {len(arrivals)} Poisson arrivals at {rate}/s over {total_s:.0f} s, "
        f"offered {offered_gpx:.3f} Gpx/s")
    main_run = serve(cfg["slots"])
    log(f"[bench] {cfg['slots']} slots: {main_run}")
    base = None
    capacity = {f"slots_{cfg['slots']}": saturate(cfg["slots"])}
    if args.served_baseline == "on":
        base = serve(1)
        log(f"[bench] 1-slot FIFO: {base}")
        capacity["fifo_one_slot"] = saturate(1)
    log(f"[bench] capacity (1000 requests at once): {capacity}")
    # offered loads above the one-slot FIFO's capacity (and below the 8-slot
    # server's), where completed frames/s can differ between the two
    loads = {}
    rates = args.served_rates
    if rates is None:
        # midway between the FIFO's and the slotted server's capacity (rounded
        # to 100/s), where the completed frames/s of the two can differ
        rates = ([round(0.5 * (capacity[f"slots_{cfg['slots']}"] + capacity["fifo_one_slot"]), -2)]
                 if "fifo_one_slot" in capacity else [])
    for hi_rate in rates:
        arr2, pk2 = trace_of(hi_rate)
        srv8 = serve(cfg["slots"], arr2, pk2)
        fifo = serve(1, arr2, pk2) if args.served_baseline == "on" else None
        loads[f"rate_{int(hi_rate)}"] = {"slots_8": srv8, "fifo_one_slot": fifo,
                                         "stable_8": bool(srv8["frames_per_s"] >= 0.95 * hi_rate),
                                         "stable_fifo": None if fifo is None else
                                         bool(fifo["frames_per_s"] >= 0.95 * hi_rate)}
        log(f"[bench] offered {hi_rate}/s: 8 slots {srv8}; FIFO {fifo}")
    # the dominant kernel as served: the trace of one 1080p request, timed and counted
    si, vi = 2, 1
    dg = pools[si][vi]
    occ = ocr.Occluders.empty(dg.height, dg.width)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        ocr.trace_occluders(bvhs[si], dg, "ao", R, None, 1, 0, occ)
    ev = _events(torch, 2)
    ev[0].record(stream)
    for s in range(10):
        ocr.trace_occluders(bvhs[si], dg, "ao", R, None, 1, s, occ)
    ev[1].record(stream)
    torch.cuda.synchronize()
    trace_ms = ev[0].elapsed_time(ev[1]) / 10
    work = counted_trace(ocr, torch, bvhs[si], dg, "ao", R, None, 1, 0)
    stable = main_run["frames_per_s"] >= 0.95 * rate
    result = {
        "metric": "frames/s and p99 frame latency, served (Poisson 400/s, 720p-1440p, AO/shadow, biased 7x7)",
        "value": main_run["frames_per_s"],
        "unit": "frames/s",
        "n_gpus": 1, "steps": main_run["requests"], "warmup": len(arrivals) - main_run["requests"],
        "ms_per_step": round(1e3 / main_run["frames_per_s"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served: 8 resident terrain scenes ({min(s.ntris for s in scenes)}.."
                               f"{max(s.ntris for s in scenes)} tris), {args.served_poses} poses x 720p/1080p/1440p "
                               f"G-buffers each, Poisson {rate}/s, {cfg['slots']} slots, "
                               f"{cfg['budget_gib']} GiB budget",
                   "global_batch": 1, "seq_len": None, "parallelism": "single-gpu"},
        "p50_ms": main_run["p50_ms"], "p99_ms": main_run["p99_ms"],
        "offered_gpx_per_s": round(offered_gpx, 3), "stable": bool(stable),
        "served": main_run, "fifo_one_slot": base, "capacity_frames_per_s": capacity, "higher_loads": loads,
        "roofline": alu_roofline(work, trace_ms, "trace_kernel (1080p request)"),
    }
    if args.cpu_baseline == "on":
        avg_px = float(np.mean([px_of[s][v] for s, v, _ in picks]))
        result["cpu_baseline"] = cpu_baseline_views(
            [scenes[2]], [(0, w.render_gbuffer(scenes[2], w.orbit_camera(2, 8, 1920, 1080)), "ao")],
            WORKLOADS["batched_16"], light, args.cpu_seconds, avg_px)
    return result


def cpu_baseline_views(scenes, views, cfg, light, budget_s, px_per_frame):
    """The oracle on 64x64-target tiles drawn from the given views (records
    for the tile's halo, then the biased 7x7 estimate) for about budget_s
    seconds; reported as frames/s of px_per_frame pixels."""
    import numpy as np

    import oracle
    oscs = [oracle.Scene(s.V, s.F) for s in scenes]
    rng = np.random.default_rng(7)
    done_px, ntiles = 0, 0
    t0 = time.perf_counter()
    while True:
        si, gb, mode = views[int(rng.integers(len(views)))]
        W, H = gb.width, gb.height
        x = int(rng.integers(0, W - 64))
        y = int(rng.integers(0, H - 64))
        t = (x, y, x + 64, y + 64)
        p = oracle.params(mode, "biased", "window", radius=cfg["window_r"], ao_radius=cfg["radius"],
                          light=light if mode == "shadow" else None, seed=1)
        rec = oracle.records(oscs[si], gb, p, oracle.halo_region(p, W, H, t))
        oracle.reuse(oscs[si], gb, p, rec, t)
        done_px += 64 * 64
        ntiles += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": round(done_px / el / px_per_frame, 5), "unit": "frames/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{ntiles} random 64x64-pixel tiles (with halos) of the workload's views, records + biased "
                      f"7x7, {el:.1f} s on {cpu_model()}; {done_px / el / 1e6:.4f} Mpx/s over "
                      f"{px_per_frame:.0f} px per frame"}


def cpu_baseline(scene, gb, cfg, light, budget_s, gpu=None):
    """The oracle, as it stands, on 64x64-target tiles of the same frame:
    records for each tile's halo, then the no-reuse, biased and unbiased
    estimates, until about budget_s seconds of work; Mrays/s = target pixels
    completed per second.  With `gpu` (the GPU's hit ids and estimates of the
    same sample), the tiles double as a parity sample: the fraction of traced
    rays the oracle flags as grazing, hit-id mismatches, and the fraction of
    targets excluded from the comparison (a differing grazing trace in the
    reuse set, or not comparable by the oracle); the others must lie within
    1e-4 of an admissible oracle value."""
    import numpy as np

    import oracle
    sc = oracle.Scene(scene.V, scene.F)
    W, H, r = gb.width, gb.height, cfg["window_r"]
    mode, R = cfg["mode"], cfg["radius"]
    mode = "shadow" if mode == "shadow2" else mode  # (the oracle takes the list of lights)
    rng = np.random.default_rng(7)
    done_px, ntiles = 0, 0
    par = dict(rays=0, grazing=0, mismatches=0, targets=0, excluded=0, compared=0, bad=0, max_err=0.0)
    t0 = time.perf_counter()
    while True:
        x = int(rng.integers(0, W - 64))
        y = int(rng.integers(0, H - 64))
        t = (x, y, x + 64, y + 64)
        pu = oracle.params(mode, "unbiased", "window", radius=r, ao_radius=R, light=light, seed=cfg["sample_seed"])
        hr = oracle.halo_region(pu, W, H, t)
        rec = oracle.records(sc, gb, pu, hr)
        res = {}
        for est in ("none", "biased", "unbiased"):
            p = oracle.params(mode, est, "window", radius=r, ao_radius=R, light=light, seed=cfg["sample_seed"])
            res[est] = oracle.reuse(sc, gb, p, rec, t)
        done_px += 64 * 64
        ntiles += 1
        if gpu is not None:
            hx0, hy0, hx1, hy1 = hr
            valid = gb.valid[hy0:hy1, hx0:hx1]
            ohit = rec.hit[hy0:hy1, hx0:hx1]
            traced = valid & (ohit != oracle.SELF)
            bad = traced & (gpu["hit"][hy0:hy1, hx0:hx1] != ohit)
            par["rays"] += int(traced.sum())
            par["grazing"] += int((traced & rec.graze[hy0:hy1, hx0:hx1].astype(bool)).sum())
            par["mismatches"] += int(bad.sum())
            # targets whose window holds a differing trace
            pad = np.pad(bad, r)
            reach = np.zeros_like(bad)
            for dy in range(2 * r + 1):
                for dx in range(2 * r + 1):
                    reach |= pad[dy:dy + bad.shape[0], dx:dx + bad.shape[1]]
            reach = reach[y - hy0:y - hy0 + 64, x - hx0:x - hx0 + 64]
            for est in ("none", "biased", "unbiased"):
                rr = res[est]
                nv = rr.nvar[y:y + 64, x:x + 64]
                if est == "none":
                    nv = np.where(bad[y - hy0:y - hy0 + 64, x - hx0:x - hx0 + 64], 0, nv)
                else:
                    nv = np.where(reach, 0, nv)
                var = rr.var[y:y + 64, x:x + 64]
                err = np.abs(gpu[est][y:y + 64, x:x + 64].astype(np.float64)[..., None] - var)
                err = np.where(np.arange(8)[None, None, :] < nv[..., None], err, np.inf).min(axis=-1)
                ok = nv > 0
                par["targets"] += int(nv.size)
                par["compared"] += int(ok.sum())
                par["excluded"] += int((~ok).sum())
                par["bad"] += int((ok & (err > 1e-4)).sum())
                if ok.any():
                    par["max_err"] = max(par["max_err"], float(err[ok].max()))
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    base = {"value": round(done_px / el / 1e6, 4), "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{ntiles} random 64x64-pixel tiles of the same frame (with their {r}-pixel halos), "
                      f"records + no-reuse + biased + unbiased 7x7, {el:.1f} s on {cpu_model()}"}
    par["tiles"] = ntiles
    par["grazing_fraction"] = round(par["grazing"] / max(1, par["rays"]), 8)
    par["excluded_fraction"] = round(par["excluded"] / max(1, par["targets"]), 8)
    par["max_err"] = float(f"{par['max_err']:.3e}")
    log(f"[bench] parity sample: {par}")
    return base, par


if __name__ == "__main__":
    main()
