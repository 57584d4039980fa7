"""Quality harness: RelMSE of the reuse estimators against a high-spp
reference on the synthetic terrain scene, the kind of evaluation of the
paper's Sec. 6 (equal-spp and equal-time tables of RelMSE ratios to no reuse,
and convergence with the sample count), with its simple baselines.

Every estimate is produced by the library's entry points on one GPU (torch
only holds buffers and evaluates the metric).  Methods, named as in the
paper (the number is the shared-group size; U = unbiased):
  RT            no reuse (one ray or segment per pixel and sample)
  Occ (N)       biased occlusion-point reuse over 2x1, 2x2, 4x2 groups
  Occ (8U)      unbiased, 4x2 groups (first-hit validation)
  Occ (7x7)     biased / unbiased over the sliding 7x7 window (this build's
  Occ (7x7U)    frame workload)
  Filter (8)    AO: final-value filtering over 4x2 groups
  Light (8)     shadows: light-sample reuse without validation (the same
                average of final values)
  Light (8U)    shadows: light-sample reuse re-traced from each target
RelMSE = mean over valid pixels of (estimate - reference)^2 / (reference^2 +
1e-3).  The reference is the mean of --ref-spp no-reuse samples (unbiased).
Sampling is white noise (the paper's low-spp comparisons use blue-noise
masks, which are not available; its convergence tests use white noise).

    python quality.py [--effects ao,shadow] [--light-sizes 1,4] [--views 3]
                      [--ref-spp 2048] [--seeds 4] [--budget-ao 2.0]
                      [--budget-shadow 5.0] [--width 1920 --height 1080]
                      [--light-pdf uniform|bilinear]

Effects: ao, shadow (area definition), shadow_sa (solid-angle definition)
and di (direct illumination of Lambertian receivers, albedo 0.8, radiance
100 / Area so that every light size emits the same power).  With
--light-pdf bilinear the light is sampled from the receiver-dependent
bilinear density (the reference stays the uniform no-reuse mean: both
estimate the same quantity); Light (8U) takes uniform sampling only and is
left out then, and for the solid-angle and DI effects.

Shadows are evaluated for each light size in --light-sizes (square lights of
that edge in metres at the benchmark light's position; 1 is the benchmark's
light, whose 12 m distance gives nearly hard shadows, larger ones give the
wide penumbrae where reuse has room to help).  MSE is reported beside
RelMSE: with epsilon = 1e-3 the latter is dominated by noise in dark pixels.

Prints one JSON line with every table, and markdown tables on stderr."""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EPS = 1e-3
R_AO = 2.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def methods(effect, pdf="uniform"):
    """name -> (kind, pattern, size, estimator)."""
    m = {"RT": ("reuse", "window", 0, "none"),
         "Occ (2)": ("reuse", "group", 2, "biased"),
         "Occ (4)": ("reuse", "group", 4, "biased"),
         "Occ (8)": ("reuse", "group", 8, "biased"),
         "Occ (8U)": ("reuse", "group", 8, "unbiased"),
         "Occ (7x7)": ("reuse", "window", 3, "biased"),
         "Occ (7x7U)": ("reuse", "window", 3, "unbiased")}
    if effect == "ao":
        m["Filter (8)"] = ("filter", "group", 8, "none")
    else:
        m["Light (8)"] = ("filter", "group", 8, "none")
        if effect == "shadow" and pdf == "uniform":
            m["Light (8U)"] = ("light", "group", 8, "none")
    return m


LIGHT_EFFECTS = ("shadow", "shadow_sa", "di")


def _reuse_light(ocr, view, p, out, ws=None, light=None):
    """The light effect's reuse entry point (records traced as shadows)."""
    light = light if light is not None else view.light
    if view.effect == "shadow_sa":
        ocr.reuse_shadow_solid_angle(view.bvh if ws is not None else None, view.dg, view.occ, light, p, out, ws)
    elif view.effect == "di":
        ocr.reuse_direct_illumination(view.bvh if ws is not None else None, view.dg, view.occ, light, p,
                                      radiance=view.radiance, albedo=0.8, out=out, workspace=ws)
    else:
        ocr.reuse_shadow(view.bvh if ws is not None else None, view.dg, view.occ, light, p, out, ws)


class View:
    def __init__(self, ocr, torch, scene, bvh, cam, effect, light):
        import workloads as w
        self.gb = w.render_gbuffer(scene, cam)
        self.dg = ocr.DeviceGBuffer.from_host(self.gb)
        self.valid = torch.from_numpy(self.gb.valid).to(self.dg.prim.device)
        self.bvh, self.effect, self.light = bvh, effect, light
        # direct illumination: the same emitted power for every light size
        self.radiance = 0.0 if light is None else 100.0 / float(
            np.linalg.norm(np.cross(light.edge_u.astype(np.float64), light.edge_v.astype(np.float64))))
        H, W = self.gb.height, self.gb.width
        dev = self.dg.prim.device
        self.occ = ocr.Occluders.empty(H, W, dev)
        self.tmp = torch.empty((H, W), dtype=torch.float32, device=dev)
        p8 = ocr.reuse_params("window", 3, 0, "unbiased")
        pg = ocr.reuse_params("group", 0, 8, "unbiased")
        self.ws = torch.empty(max(ocr.workspace_bytes(W, H, p8), ocr.workspace_bytes(W, H, pg)), dtype=torch.uint8,
                              device=dev)


def run_sample(ocr, view, spec, seed, sample, out, accumulate, light=None):
    """Enqueue one sample of a method, writing (or adding to) out (light:
    another sampling of the view's light, e.g. for the reference)."""
    kind, pattern, size, est = spec
    light = light if light is not None else view.light
    if kind == "light":
        p = ocr.reuse_params(pattern, size, size, "none", accumulate=accumulate)
        ocr.light_reuse_shadow(view.bvh, view.dg, light, seed, sample, p, out)
        return
    tmode = "ao" if view.effect == "ao" else "shadow"
    ocr.trace_occluders(view.bvh, view.dg, tmode, R_AO, light, seed, sample, view.occ)
    if kind == "filter":
        p = ocr.reuse_params("window", 0, 0, "none")
        if view.effect == "ao":
            ocr.reuse_ao(None, view.dg, view.occ, R_AO, p, view.tmp)
        else:
            _reuse_light(ocr, view, p, view.tmp, light=light)
        ocr.filter_values(view.dg, ocr.reuse_params(pattern, size, size, "none", accumulate=accumulate), view.tmp,
                          out)
        return
    p = ocr.reuse_params(pattern, size, size, est, accumulate=accumulate)
    if view.effect == "ao":
        ocr.reuse_ao(view.bvh, view.dg, view.occ, R_AO, p, out, view.ws)
    else:
        _reuse_light(ocr, view, p, out, view.ws, light=light)


def render(ocr, torch, view, spec, seed, nspp, first=0, light=None):
    out = torch.empty_like(view.tmp)
    for s in range(nspp):
        run_sample(ocr, view, spec, seed, first + s, out, s > 0, light)
    if nspp > 1:
        ocr.scale(out, 1.0 / nspp)
    return out


def relmse(torch, est, ref, valid):
    d = (est - ref) ** 2 / (ref * ref + EPS)
    return float(d[valid].mean().item())


def mse(torch, est, ref, valid):
    return float(((est - ref) ** 2)[valid].mean().item())


def square_light(w, size, pdf=0):
    base = w.terrain_light()
    return w.RectLight(base.center.copy(), base.edge_u * size, base.edge_v * size, pdf)


def time_per_spp(ocr, torch, view, spec, reps=5):
    out = torch.empty_like(view.tmp)
    for s in range(2):
        run_sample(ocr, view, spec, 77, s, out, False)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for s in range(reps):
        run_sample(ocr, view, spec, 78, s, out, s > 0)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def evaluate(ocr, torch, effect, args, light_size=1.0):
    import numpy as np

    import workloads as w
    scene = w.terrain_scene(2)
    bvh = ocr.build_bvh(scene.V, scene.F)
    pdf = 1 if args.light_pdf == "bilinear" else 0
    light = square_light(w, light_size, pdf) if effect in LIGHT_EFFECTS else None
    ref_light = square_light(w, light_size) if effect in LIGHT_EFFECTS else None
    W, H = args.width, args.height
    cams = [w.terrain_camera(W, H)] + [w.orbit_camera(v, args.views, W, H) for v in range(1, args.views)]
    ms = methods(effect, args.light_pdf)
    budget = args.budget_ao if effect == "ao" else args.budget_shadow
    per_view = []
    times = None
    for vi, cam in enumerate(cams):
        view = View(ocr, torch, scene, bvh, cam, effect, light)
        t0 = time.time()
        ref = render(ocr, torch, view, ms["RT"], 999, args.ref_spp, light=ref_light)
        torch.cuda.synchronize()
        log(f"[quality] {effect} view {vi}: reference {args.ref_spp} spp in {time.time() - t0:.1f} s, "
            f"valid {view.gb.valid.mean():.3f}, mean {float(ref[view.valid].mean()):.4f}")
        if times is None:
            times = {n: time_per_spp(ocr, torch, view, spec) for n, spec in ms.items()}
        eq_spp, eq_mse = {}, {}
        for n, spec in ms.items():
            outs = [render(ocr, torch, view, spec, 1 + k, 1) for k in range(args.seeds)]
            eq_spp[n] = float(np.mean([relmse(torch, o, ref, view.valid) for o in outs]))
            eq_mse[n] = float(np.mean([mse(torch, o, ref, view.valid) for o in outs]))
        eq_time, spp = {}, {}
        for n, spec in ms.items():
            spp[n] = max(1, int(math.floor(budget / times[n])))
            errs = [relmse(torch, render(ocr, torch, view, spec, 101 + k, spp[n]), ref, view.valid)
                    for k in range(max(1, args.seeds // 2))]
            eq_time[n] = float(np.mean(errs))
        per_view.append(dict(equal_spp=eq_spp, equal_spp_mse=eq_mse, equal_time=eq_time, spp=spp))
        if vi == 0:
            conv = {}
            for n in ("RT", "Occ (8)", "Occ (8U)", "Occ (7x7)", "Occ (7x7U)"):
                conv[n] = {k: relmse(torch, render(ocr, torch, view, ms[n], 201, k), ref, view.valid)
                           for k in (1, 4, 16, 64)}
        del view
    names = list(ms)

    def ratios(key):
        return {n: float(np.mean([v[key][n] / v[key]["RT"] for v in per_view])) for n in names}

    return dict(effect=effect, light_m=light_size if effect in LIGHT_EFFECTS else None, light_pdf=args.light_pdf,
                views=len(cams), size=f"{W}x{H}",
                ref_spp=args.ref_spp, seeds=args.seeds,
                budget_ms=budget, ms_per_spp={n: round(times[n], 4) for n in names},
                equal_spp_relmse={n: float(np.mean([v["equal_spp"][n] for v in per_view])) for n in names},
                equal_spp_ratio=ratios("equal_spp"), equal_spp_mse_ratio=ratios("equal_spp_mse"),
                equal_time_spp={n: per_view[0]["spp"][n] for n in names},
                equal_time_relmse={n: float(np.mean([v["equal_time"][n] for v in per_view])) for n in names},
                equal_time_ratio=ratios("equal_time"),
                convergence={n: {str(k): v for k, v in c.items()} for n, c in conv.items()})


def markdown(res):
    names = list(res["ms_per_spp"])
    light = f", {res['light_m']:g} m light, {res['light_pdf']} density" if res["light_m"] else ""
    lines = [f"### {res['effect']} ({res['size']}{light}, {res['views']} views, reference {res['ref_spp']} spp)", "",
             "| method | ms/spp | equal-spp RelMSE | ratio | MSE ratio | equal-time spp | equal-time RelMSE | ratio |",
             "|---|---|---|---|---|---|---|---|"]
    for n in names:
        lines.append(f"| {n} | {res['ms_per_spp'][n]:.3f} | {res['equal_spp_relmse'][n]:.4f} | "
                     f"{res['equal_spp_ratio'][n]:.2f}x | {res['equal_spp_mse_ratio'][n]:.2f}x | "
                     f"{res['equal_time_spp'][n]} | {res['equal_time_relmse'][n]:.4f} | "
                     f"{res['equal_time_ratio'][n]:.2f}x |")
    lines += ["", "| convergence (view 0) | 1 spp | 4 | 16 | 64 |", "|---|---|---|---|---|"]
    for n, c in res["convergence"].items():
        lines.append(f"| {n} | " + " | ".join(f"{c[k]:.4f}" for k in ("1", "4", "16", "64")) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--effects", default="ao,shadow")
    ap.add_argument("--light-sizes", default="1,4")
    ap.add_argument("--views", type=int, default=3)
    ap.add_argument("--ref-spp", type=int, default=2048)
    ap.add_argument("--seeds", type=int, default=4)
    ap.add_argument("--budget-ao", type=float, default=2.0)
    ap.add_argument("--budget-shadow", type=float, default=5.0)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--light-pdf", default="uniform", choices=["uniform", "bilinear"])
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        sys.exit("quality.py needs a GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    out = {}
    for effect in args.effects.split(","):
        sizes = [float(v) for v in args.light_sizes.split(",")] if effect in LIGHT_EFFECTS else [1.0]
        for size in sizes:
            res = evaluate(ocr, torch, effect, args, size)
            log(markdown(res))
            out[effect if effect == "ao" else f"{effect}_{size:g}m"] = res
    print(json.dumps(out))


if __name__ == "__main__":
    main()
