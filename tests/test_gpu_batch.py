"""Batched schedule on the GPU: one plan over many views of uneven size,
several scenes and mixed AO, shadows, solid-angle shadows and direct
illumination, estimators and patterns.

Each view's records and estimate must be bitwise identical to the per-view
entry points with the same arguments (which the parity tests hold to the
oracle), for every tile and packing knob, with and without the HIP graph,
and on every replay of the graph; two views are also compared with the
oracle directly, and the full sixteen-view workload is checked at size."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_util import compare_values, log, mismatch_reach, tiles, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TILES = [(8, 8), (16, 8), (16, 16), (32, 8), (32, 16)]


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


BOX_LIGHT = w.RectLight(np.array([0.0, 6.0, 0.0], np.float32), np.array([2.0, 0.0, 0.0], np.float32),
                        np.array([0.0, 0.0, 2.0], np.float32))

# (scene, W, H, mode, pattern, size, estimator, dark_guard)
SPECS = [(0, 61, 37, "ao", "window", 2, "biased", True),
         (1, 96, 64, "shadow", "window", 3, "biased", True),
         (0, 130, 70, "shadow", "window", 4, "unbiased", True),
         (1, 45, 90, "ao", "window", 3, "unbiased", True),
         (1, 200, 113, "ao", "window", 3, "none", True),
         (0, 33, 17, "ao", "group", 8, "biased", True),
         (1, 100, 60, "shadow", "group", 4, "unbiased", True),
         (0, 1, 1, "ao", "window", 2, "biased", True),
         (1, 64, 64, "shadow", "window", 8, "biased", False),
         (0, 77, 41, "shadow_sa", "window", 3, "biased", True),
         (1, 90, 50, "shadow_sa", "window", 2, "unbiased", True),
         (0, 40, 40, "shadow_sa", "group", 8, "unbiased", True),
         (1, 120, 64, "di", "window", 3, "biased", True),
         (0, 64, 48, "di", "window", 3, "unbiased", True),
         (1, 50, 30, "di", "window", 2, "none", True),
         (0, 36, 20, "di", "group", 4, "biased", True),
         (1, 70, 31, "shadow_sa", "window", 3, "none", True)]
DI_RADIANCE, DI_ALBEDO = 50.0, 0.7


class View:
    pass


@pytest.fixture(scope="module")
def mixed(ocr):
    scenes = [w.boxes_scene(1), w.terrain_scene(seed=10, cells=64, nspheres=20)]
    bvhs = [ocr.build_bvh(s.V, s.F) for s in scenes]
    lights = [BOX_LIGHT, w.terrain_light()]
    views = []
    for i, (si, W, H, mode, pattern, size, est, guard) in enumerate(SPECS):
        v = View()
        cam = w.boxes_camera(W, H) if si == 0 else w.orbit_camera(i, len(SPECS), W, H)
        v.si, v.mode, v.W, v.H = si, mode, W, H
        v.gb = w.render_gbuffer(scenes[si], cam)
        v.dg = ocr.DeviceGBuffer.from_host(v.gb)
        v.R = 1.0 if si == 0 else 2.0
        v.light = lights[si] if mode != "ao" else None
        v.seed, v.sample = 100 + i, i % 3
        v.params = ocr.reuse_params(pattern, size, size, est, dark_guard=guard)
        v.opattern, v.osize, v.oest, v.oguard = pattern, size, est, guard
        # the per-view reference
        occ = ocr.trace_occluders(bvhs[si], v.dg, "ao" if mode == "ao" else "shadow", v.R, v.light, v.seed,
                                  v.sample)
        if mode == "ao":
            ref = ocr.reuse_ao(bvhs[si], v.dg, occ, v.R, v.params)
        elif mode == "shadow":
            ref = ocr.reuse_shadow(bvhs[si], v.dg, occ, v.light, v.params)
        elif mode == "shadow_sa":
            ref = ocr.reuse_shadow_solid_angle(bvhs[si], v.dg, occ, v.light, v.params)
        else:
            ref = ocr.reuse_direct_illumination(bvhs[si], v.dg, occ, v.light, v.params, radiance=DI_RADIANCE,
                                                albedo=DI_ALBEDO)
        torch.cuda.synchronize()
        v.ref_out = to_np(ref).copy()
        v.ref_hit = occ.hit_u32().copy()
        v.ref_dz, v.ref_nz = to_np(occ.dz).copy(), to_np(occ.nz).copy()
        views.append(v)
    return scenes, bvhs, views


def _descs(ocr, bvhs, views):
    outs = [torch.full((v.H, v.W), float("nan"), dtype=torch.float32, device="cuda") for v in views]
    descs = [ocr.view_desc(bvhs[v.si], v.dg, outs[i], v.mode, v.R, v.light, v.seed, v.sample, v.params,
                           radiance=DI_RADIANCE, albedo=DI_ALBEDO) for i, v in enumerate(views)]
    return descs, outs


def _check_plan(ocr, plan, views, outs, what):
    torch.cuda.synchronize()
    for i, v in enumerate(views):
        got = to_np(outs[i])
        assert np.array_equal(got.view(np.uint32), v.ref_out.view(np.uint32)), (what, i)
        dz, nz, hit = plan.records_host(i, v.H, v.W)
        assert np.array_equal(hit, v.ref_hit), (what, i)
        m = v.ref_hit < oracle.SELF
        assert np.array_equal(dz[m].view(np.uint32), v.ref_dz[m].view(np.uint32)), (what, i)
        assert np.array_equal(nz[m].view(np.uint32), v.ref_nz[m].view(np.uint32)), (what, i)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_plan_bitwise_equals_per_view_every_knob(ocr, mixed, use_graph):
    _, bvhs, views = mixed
    for tw, th in TILES:
        for pack in ("row", "block8", "morton"):
            log(f"[plan] tile {tw}x{th} {pack} graph={use_graph}")
            descs, outs = _descs(ocr, bvhs, views)
            plan = ocr.Plan(descs, ocr.plan_tuning((tw, th), pack, use_graph))
            plan.launch()
            _check_plan(ocr, plan, views, outs, (tw, th, pack, use_graph))
            info = plan.info()
            assert info.nviews == len(views) and info.tuned == 0
            assert info.pixels == sum(v.W * v.H for v in views)
            plan.free()


def test_plan_autotune(ocr, mixed):
    _, bvhs, views = mixed
    log("[plan] autotune")
    descs, outs = _descs(ocr, bvhs, views)
    plan = ocr.Plan(descs)
    info = plan.info()
    assert info.tuned == 1 and info.candidates == 13 and info.best_trace_ms > 0
    assert (info.tuning.tile_w, info.tuning.tile_h) in TILES and info.tuning.use_graph == 1
    plan.launch()
    _check_plan(ocr, plan, views, outs, "autotuned")
    plan.free()


def test_plan_autotune_choice_is_kept(ocr, mixed):
    # a second autotuned plan over views of the same shape takes the first
    # plan's choice without timing, and computes the same bits
    _, bvhs, views = mixed
    log("[plan] autotune twice")
    descs, outs = _descs(ocr, bvhs, views)
    p1 = ocr.Plan(descs)
    i1 = p1.info()
    p1.launch()
    torch.cuda.synchronize()
    out1 = [to_np(o).copy() for o in outs]
    p1.free()
    p2 = ocr.Plan(descs)
    i2 = p2.info()
    assert i2.tuned == 1 and i2.from_cache == 1 and i2.candidates == 0
    assert (i2.tuning.tile_w, i2.tuning.tile_h, i2.tuning.packing) == (i1.tuning.tile_w, i1.tuning.tile_h,
                                                                      i1.tuning.packing)
    p2.launch()
    _check_plan(ocr, p2, views, outs, "cached tuning")
    for o, o1 in zip(outs, out1):
        assert np.array_equal(to_np(o).view(np.uint32), o1.view(np.uint32))
    p2.free()


def test_plan_graph_replays(ocr, mixed):
    # replay several times with the program's own eager work and
    # synchronisations between replays; every replay must reproduce the result
    _, bvhs, views = mixed
    descs, outs = _descs(ocr, bvhs, views)
    plan = ocr.Plan(descs, ocr.plan_tuning((32, 8), "morton", True))
    for rep in range(4):
        log(f"[plan] graph replay {rep}")
        for o in outs:
            o.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work on the same stream
        plan.launch()
        junk = junk + torch.ones(8, device="cuda").sum()
        torch.cuda.synchronize()
        _check_plan(ocr, plan, views, outs, f"replay {rep}")
    plan.free()


def test_plan_views_against_oracle(ocr, mixed):
    scenes, bvhs, views = mixed
    descs, outs = _descs(ocr, bvhs, views)
    plan = ocr.Plan(descs, ocr.plan_tuning((16, 16), "block8", True))
    plan.launch()
    torch.cuda.synchronize()
    for i in (0, 1, 3, 9, 12):
        v = views[i]
        log(f"[plan vs oracle] view {i}: {v.W}x{v.H} {v.mode} {v.opattern} {v.osize} {v.oest}")
        p = oracle.params(v.mode, v.oest, v.opattern, radius=v.osize, group_n=v.osize, dark_guard=v.oguard,
                          ao_radius=v.R, light=v.light, seed=v.seed, sample=v.sample)
        osc = oracle.Scene(scenes[v.si].V, scenes[v.si].F)
        rec, res = oracle.frame(osc, v.gb, p)
        if v.mode == "di":
            # the oracle works in units of albedo * radiance / pi
            k = DI_ALBEDO * DI_RADIANCE / np.pi
            res.value, res.var = res.value * k, res.var * k
        _, _, hit = plan.records_host(i, v.H, v.W)
        st = compare_values(to_np(outs[i]), res, exclude=mismatch_reach(hit, rec, p))
        log(f"    {st}")
    plan.free()


def test_plan_argument_errors(ocr, mixed):
    _, bvhs, views = mixed
    descs, outs = _descs(ocr, bvhs, views[:2])
    with pytest.raises(ocr.OcrError) as e:
        ocr.Plan(descs, ocr.plan_tuning((24, 8), "row", True))
    assert e.value.status == -1
    with pytest.raises(ocr.OcrError):
        ocr.Plan(descs, ocr.PlanTuning(16, 16, 7, 1))
    bad = list(descs)
    bad[1].params = ocr.reuse_params("window", 3, 0, "biased", accumulate=True)
    with pytest.raises(ocr.OcrError):
        ocr.Plan(bad, ocr.plan_tuning())
    bad[1].params = ocr.reuse_params("window", 3, 0, "biased")
    bad[1].ao_radius = float("nan")
    bad[1].mode = 0
    with pytest.raises(ocr.OcrError):
        ocr.Plan(bad, ocr.plan_tuning())
    with pytest.raises(ocr.OcrError):
        ocr.Plan([], ocr.plan_tuning())
    # an unknown mode, a negative radiance, and a light of another density
    bad = list(_descs(ocr, bvhs, views[1:3])[0])
    bad[0].mode = 7
    with pytest.raises(ocr.OcrError):
        ocr.Plan(bad, ocr.plan_tuning())
    bad[0].mode = 3
    bad[0].radiance = -1.0
    with pytest.raises(ocr.OcrError):
        ocr.Plan(bad, ocr.plan_tuning())
    bad[0].radiance = 1.0
    bad[0].light.pdf = 1
    with pytest.raises(ocr.OcrError) as e:
        ocr.Plan(bad, ocr.plan_tuning())
    assert e.value.status == -4


def test_batched_workload_full_size(ocr):
    """The sixteen-view, four-scene workload the benchmark times, autotuned:
    bitwise equal to sixteen per-view launch pairs, and sampled tiles of one
    AO and one shadow view against the oracle."""
    scenes = []
    for i in range(4):
        log(f"[batched 16] scene {i}")
        scenes.append(w.batch_scene(i))
    bvhs = [ocr.build_bvh(s.V, s.F) for s in scenes]
    light = w.terrain_light()
    params = ocr.reuse_params("window", 3, 0, "biased")
    vs = []
    for v, (si, cam, mode) in enumerate(w.batch_views()):
        gb = w.render_gbuffer(scenes[si], cam)
        vs.append((si, gb, ocr.DeviceGBuffer.from_host(gb), mode))
    log(f"[batched 16] {sum(g.width * g.height for _, g, _, _ in vs)} px")
    outs, descs, refs = [], [], []
    for v, (si, gb, dg, mode) in enumerate(vs):
        lt = light if mode == "shadow" else None
        occ = ocr.trace_occluders(bvhs[si], dg, mode, 2.0, lt, 1, 0)
        r = ocr.reuse_ao(bvhs[si], dg, occ, 2.0, params) if mode == "ao" else \
            ocr.reuse_shadow(bvhs[si], dg, occ, light, params)
        torch.cuda.synchronize()
        refs.append((to_np(r).copy(), occ.hit_u32().copy()))
        o = torch.full((gb.height, gb.width), float("nan"), dtype=torch.float32, device="cuda")
        outs.append(o)
        descs.append(ocr.view_desc(bvhs[si], dg, o, mode, 2.0, lt, 1, 0, params))
    plan = ocr.Plan(descs)
    info = plan.info()
    log(f"[batched 16] tuned tile {info.tuning.tile_w}x{info.tuning.tile_h} packing {info.tuning.packing} "
        f"trace {info.best_trace_ms:.3f} ms, tune {info.tune_ms:.0f} ms")
    plan.launch()
    torch.cuda.synchronize()
    for v, (si, gb, dg, mode) in enumerate(vs):
        assert np.array_equal(to_np(outs[v]).view(np.uint32), refs[v][0].view(np.uint32)), v
        _, _, hit = plan.records_host(v, gb.height, gb.width)
        assert np.array_equal(hit, refs[v][1]), v
    for v in (8, 3):  # AO on the 1.16M-triangle scene; shadow on the 2M-triangle one
        si, gb, dg, mode = vs[v]
        osc = oracle.Scene(scenes[si].V, scenes[si].F)
        p = oracle.params(mode, "biased", "window", radius=3, ao_radius=2.0,
                          light=light if mode == "shadow" else None, seed=1, sample=0)
        gpu = to_np(outs[v])
        for t in tiles(gb.width, gb.height, 3, 32, seed=20 + v):
            hr = oracle.halo_region(p, gb.width, gb.height, t)
            rec = oracle.records(osc, gb, p, hr)
            res = oracle.reuse(osc, gb, p, rec, t)
            inside = np.zeros_like(gb.valid)
            inside[hr[1]:hr[3], hr[0]:hr[2]] = True
            st = compare_values(gpu, res, region=t, exclude=mismatch_reach(np.where(inside, refs[v][1], rec.hit),
                                                                           rec, p))
            log(f"    view {v} tile {t}: {st}")
    plan.free()


def test_plan_without_window_views(ocr, mixed):
    # only fixed-group and no-reuse views: no batched window reuse launch (group views go per view)
    _, bvhs, views = mixed
    sub = [v for v in views if v.opattern == "group" or v.oest == "none"]
    assert len(sub) >= 3
    for use_graph in (0, 1):
        log(f"[plan] group / no-reuse views only, graph={use_graph}")
        descs, outs = _descs(ocr, bvhs, sub)
        plan = ocr.Plan(descs, ocr.plan_tuning((8, 8), "row", use_graph))
        plan.launch()
        plan.launch()
        _check_plan(ocr, plan, sub, outs, f"group-only graph={use_graph}")
        plan.free()
