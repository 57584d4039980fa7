"""GPU parity of shadows of several rectangular lights (the oracle's reading:
the visible fraction of the total emitting area, each sample on light l with
probability A_l / A_tot, densities summed over the lights), through the C-ABI.

One light given as a list is bitwise the single-light path; with two lights
(one of them rotated and tilted, so that the FP32 light terms are not exact)
the records match the oracle's (hit ids, except flagged grazing rays) and the
estimates lie within 1e-4 of an admissible oracle value."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_util import compare_hits, compare_values, log, mismatch_reach, tiles, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


def _lights():
    return w.two_lights()


class Case:
    def __init__(self, ocr, name, scene, gb):
        log(f"[case] {name}: {gb.width}x{gb.height}, {scene.ntris} tris")
        self.scene, self.gb = scene, gb
        self.bvh = ocr.build_bvh(scene.V, scene.F)
        self.dg = ocr.DeviceGBuffer.from_host(gb)
        self.osc = oracle.Scene(scene.V, scene.F)


@pytest.fixture(scope="module")
def terrain_small(ocr):
    s = w.terrain_scene(2)
    return Case(ocr, "terrain_480x270", s, w.render_gbuffer(s, w.terrain_camera(480, 270)))


def test_one_light_list_is_the_single_light(ocr, terrain_small):
    case, light = terrain_small, w.terrain_light()
    a = ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, light, 4, 1)
    b = ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, [light], 4, 1)
    torch.cuda.synchronize()
    assert np.array_equal(a.hit_u32(), b.hit_u32())
    assert np.array_equal(to_np(a.dz).view(np.uint32), to_np(b.dz).view(np.uint32))
    for est in ("none", "biased", "unbiased"):
        p = ocr.reuse_params("window", 3, 0, est)
        x = to_np(ocr.reuse_shadow(case.bvh, case.dg, a, light, p))
        y = to_np(ocr.reuse_shadow(case.bvh, case.dg, a, [light], p))
        torch.cuda.synchronize()
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), est


def test_two_light_records_match_oracle(ocr, terrain_small):
    case, lights = terrain_small, _lights()
    occ = ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, lights, 7, 3)
    torch.cuda.synchronize()
    rec = oracle.records(case.osc, case.gb, oracle.params("shadow", "none", light=lights, seed=7, sample=3))
    st = compare_hits(occ.hit_u32(), rec, case.gb.valid)
    log(f"    {st}")
    # both lights are sampled: the hits and self-blocked samples of each
    hit = occ.hit_u32()[case.gb.valid]
    assert (hit < oracle.SELF).any() and (hit == oracle.MISS).any()


@pytest.mark.parametrize("pattern,size,est", [("window", 3, "biased"), ("window", 2, "unbiased"),
                                              ("window", 3, "unbiased"), ("group", 8, "biased"),
                                              ("group", 4, "unbiased"), ("window", 3, "none")])
def test_two_light_reuse_matches_oracle(ocr, terrain_small, pattern, size, est):
    case, lights = terrain_small, _lights()
    log(f"[two lights 480x270] {pattern} {size} {est}")
    occ = ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, lights, 3, 0)
    gpu = to_np(ocr.reuse_shadow(case.bvh, case.dg, occ, lights, ocr.reuse_params(pattern, size, size, est)))
    torch.cuda.synchronize()
    p = oracle.params("shadow", est, pattern, radius=size, group_n=size, light=lights, seed=3)
    rec, res = oracle.frame(case.osc, case.gb, p)
    st = compare_values(gpu, res, exclude=mismatch_reach(occ.hit_u32(), rec, p))
    log(f"    {st}")


@pytest.mark.parametrize("est,ntiles", [("biased", 6), ("unbiased", 3)])
def test_two_light_1080p_tiles(ocr, est, ntiles):
    s = w.terrain_scene(2)
    case = Case(ocr, "terrain_1080p", s, w.render_gbuffer(s, w.terrain_camera()))
    lights = _lights()
    occ = ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, lights, 1, 0)
    gpu = to_np(ocr.reuse_shadow(case.bvh, case.dg, occ, lights, ocr.reuse_params("window", 3, 0, est)))
    torch.cuda.synchronize()
    assert np.isfinite(gpu).all() and (gpu[~case.gb.valid] == 0.0).all()
    p = oracle.params("shadow", est, "window", radius=3, light=lights, seed=1)
    gh = occ.hit_u32()
    for t in tiles(case.gb.width, case.gb.height, ntiles, 32, seed=31):
        hr = oracle.halo_region(p, case.gb.width, case.gb.height, t)
        rec = oracle.records(case.osc, case.gb, p, hr)
        res = oracle.reuse(case.osc, case.gb, p, rec, t)
        inside = np.zeros_like(case.gb.valid)
        inside[hr[1]:hr[3], hr[0]:hr[2]] = True
        st = compare_values(gpu, res, region=t, exclude=mismatch_reach(np.where(inside, gh, rec.hit), rec, p))
        log(f"    tile {t}: {st}")


def test_light_count_errors(ocr, terrain_small):
    case = terrain_small
    occ = ocr.Occluders.empty(case.gb.height, case.gb.width)
    with pytest.raises(ocr.OcrError):
        ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, [w.terrain_light()] * 5, 1, 0, occ)
    with pytest.raises(ValueError):
        ocr.trace_occluders(case.bvh, case.dg, "ao", 1.0, [w.terrain_light()], 1, 0, occ)
