"""GPU parity of lights sampled from the general (bilinear, receiver-dependent)
emitter-area density, through the C-ABI: samples bit-exact, records equal to
the oracle's but for flagged grazing rays, and shadows (area and solid-angle
definitions) and direct illumination within 1e-4 of an admissible oracle
value, on the terrain under a large low light and on tilted receivers close
to a light (where the density varies most)."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w
from gpu_util import compare_hits, compare_values, log, mismatch_reach, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# direct illumination with albedo pi: the GPU's value is the oracle's (in
# units of rho L_e / pi) times the radiance
DI_ALBEDO = float(np.pi)


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


class Case:
    def __init__(self, ocr, name, scene, gb, light):
        log(f"[case] {name}: {gb.width}x{gb.height}, {scene.ntris} tris")
        self.name, self.scene, self.gb, self.light = name, scene, gb, light
        self.bvh = ocr.build_bvh(scene.V, scene.F)
        self.dg = ocr.DeviceGBuffer.from_host(gb)
        self.osc = oracle.Scene(scene.V, scene.F)


def _low_light(pdf=1):
    # 4 x 4 m, 2.5 m above the highest terrain point (terrain_light's centre)
    return w.RectLight(np.array([0.0, 6.5, 12.0], np.float32), np.array([4.0, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, 4.0], np.float32), pdf)


@pytest.fixture(scope="module")
def terrain(ocr):
    s = w.terrain_scene(2)
    return Case(ocr, "terrain_480x270_low_light", s, w.render_gbuffer(s, w.terrain_camera(480, 270)), _low_light())


@pytest.fixture(scope="module")
def near(ocr):
    # tilted receivers 1 m below a light, under a high plate and a low strip
    s = scenes.build([scenes.FLOOR, scenes.plate_y(0.5, -0.5, 0.02, -3, 3), scenes.plate_y(0.1, -0.12, -0.06, -3, 3)])
    gb = scenes.floor_grid(96, 64, 0.01, x0=-0.5, z0=-0.3)
    th = np.arctan2(1.0, -0.1)
    gb.nrm[:] = np.array([np.sin(th), np.cos(th), 0.0], np.float32)
    light = w.RectLight(np.array([0.2, 1.0, 0.1], np.float32), np.array([1.2, 0, 0], np.float32),
                        np.array([0, 0, 1.2], np.float32), 1)
    return Case(ocr, "tilted_near_light", s, gb, light)


def _trace(ocr, case, seed, sample=0, light=None):
    occ = ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, light or case.light, seed, sample)
    torch.cuda.synchronize()
    return occ


def _reuse(ocr, case, mode, occ, params, light=None, radiance=1.0):
    light = light or case.light
    if mode == "shadow_sa":
        out = ocr.reuse_shadow_solid_angle(case.bvh, case.dg, occ, light, params)
    elif mode == "di":
        out = ocr.reuse_direct_illumination(case.bvh, case.dg, occ, light, params, radiance=radiance,
                                            albedo=DI_ALBEDO)
    else:
        out = ocr.reuse_shadow(case.bvh, case.dg, occ, light, params)
    torch.cuda.synchronize()
    return to_np(out)


@pytest.mark.parametrize("which", ["terrain", "near"])
def test_samples_bit_exact(ocr, request, which):
    case = request.getfixturevalue(which)
    for seed, sample in [(1, 0), (0xDEADBEEF12345678, 7)]:
        log(f"[bilinear samples] {case.name} seed={seed} sample={sample}")
        o, d, k = ocr.sample_rays(case.dg, "shadow", case.light, seed, sample)
        torch.cuda.synchronize()
        ro, rd, rk = oracle.samples(case.gb, oracle.params("shadow", "none", light=case.light, seed=seed,
                                                          sample=sample))
        assert np.array_equal(to_np(k), rk)
        assert np.array_equal(to_np(o).view(np.uint32), ro.view(np.uint32))
        assert np.array_equal(to_np(d).view(np.uint32), rd.view(np.uint32))
    # the density is not the uniform one: the same hashes give other points
    _, du, _ = ocr.sample_rays(case.dg, "shadow", _low_light(0) if which == "terrain" else
                               w.RectLight(case.light.center, case.light.edge_u, case.light.edge_v), 1, 0)
    _, db, _ = ocr.sample_rays(case.dg, "shadow", case.light, 1, 0)
    torch.cuda.synchronize()
    assert (to_np(du) != to_np(db)).any(axis=-1).mean() > 0.5


@pytest.mark.parametrize("which", ["terrain", "near"])
def test_records_match_oracle(ocr, request, which):
    case = request.getfixturevalue(which)
    log(f"[bilinear records] {case.name}")
    occ = _trace(ocr, case, 5, 2)
    rec = oracle.records(case.osc, case.gb, oracle.params("shadow", "none", light=case.light, seed=5, sample=2))
    st = compare_hits(occ.hit_u32(), rec, case.gb.valid)
    log(f"    {st}")
    hit = occ.hit_u32()[case.gb.valid]
    assert (hit < oracle.SELF).any() and (hit == oracle.MISS).any()


CONFIGS = [("window", 3, "biased"), ("window", 2, "unbiased"), ("window", 3, "unbiased"), ("group", 8, "biased"),
           ("group", 4, "unbiased"), ("window", 3, "none")]


@pytest.mark.parametrize("mode", ["shadow", "shadow_sa", "di"])
@pytest.mark.parametrize("pattern,size,est", CONFIGS)
def test_terrain_reuse_matches_oracle(ocr, terrain, mode, pattern, size, est):
    case = terrain
    log(f"[bilinear {mode} 480x270] {pattern} {size} {est}")
    # direct illumination: a radiance of 100 puts the values near 1
    k = 100.0 if mode == "di" else 1.0
    occ = _trace(ocr, case, 3)
    gpu = _reuse(ocr, case, mode, occ, ocr.reuse_params(pattern, size, size, est), radiance=k)
    p = oracle.params(mode, est, pattern, radius=size, group_n=size, light=case.light, seed=3)
    rec, res = oracle.frame(case.osc, case.gb, p)
    res.value, res.var = res.value * k, res.var * k
    st = compare_values(gpu, res, exclude=mismatch_reach(occ.hit_u32(), rec, p))
    log(f"    {st}")


@pytest.mark.parametrize("mode", ["shadow", "shadow_sa", "di"])
@pytest.mark.parametrize("pattern,size,est", [("window", 0, "none"), ("window", 2, "biased"), ("window", 2, "unbiased"),
                                              ("group", 8, "unbiased")])
def test_near_light_reuse_matches_oracle(ocr, near, mode, pattern, size, est):
    case = near
    log(f"[bilinear {mode} near light] {pattern} {size} {est}")
    k = 4.0 if mode == "di" else 1.0
    occ = _trace(ocr, case, 6)
    gpu = _reuse(ocr, case, mode, occ, ocr.reuse_params(pattern, size, size, est), radiance=k)
    p = oracle.params(mode, est, pattern, radius=size, group_n=size, light=case.light, seed=6)
    rec, res = oracle.frame(case.osc, case.gb, p)
    res.value, res.var = res.value * k, res.var * k
    # the plates' edges lie on pixel columns of this grid, so more segments
    # graze them than on the terrain (the oracle flags those targets)
    st = compare_values(gpu, res, exclude=mismatch_reach(occ.hit_u32(), rec, p), max_excluded=1e-2)
    log(f"    {st}")


def test_the_density_enters_the_estimate(ocr, terrain):
    # the same records reused as if sampled uniformly give other values
    case = terrain
    occ = _trace(ocr, case, 3)
    p = ocr.reuse_params("window", 3, 0, "biased")
    a = _reuse(ocr, case, "shadow", occ, p)
    b = _reuse(ocr, case, "shadow", occ, p, light=_low_light(0))
    v = case.gb.valid & (occ.hit_u32() < oracle.SELF)
    assert np.abs(a - b)[v].max() > 0.05


def test_entry_points_that_sample_uniformly_refuse_it(ocr, terrain):
    case = terrain
    occ = ocr.Occluders.empty(case.gb.height, case.gb.width)
    with pytest.raises(ocr.OcrError):
        ocr.trace_occluders(case.bvh, case.dg, "shadow", 1.0, [case.light, _low_light(0)], 1, 0, occ)
    with pytest.raises(ocr.OcrError):
        ocr.light_reuse_shadow(case.bvh, case.dg, case.light, 1, 0, ocr.reuse_params("window", 1, 0, "biased"))
    assert b"uniformly" in ocr.lib().ocr_last_error()


@pytest.mark.parametrize("est,ntiles", [("biased", 6), ("unbiased", 3)])
def test_solid_angle_1080p_tiles(ocr, est, ntiles):
    # the benchmark's configuration: 1080p terrain, the 1 m light sampled from
    # the bilinear density, solid-angle shadows, 7x7 window; sampled tiles
    from gpu_util import tiles
    s = w.terrain_scene(2)
    light = w.terrain_light()
    light.pdf = 1
    case = Case(ocr, "terrain_1080p", s, w.render_gbuffer(s, w.terrain_camera()), light)
    occ = _trace(ocr, case, 1)
    gpu = _reuse(ocr, case, "shadow_sa", occ, ocr.reuse_params("window", 3, 0, est))
    assert np.isfinite(gpu).all() and (gpu[~case.gb.valid] == 0.0).all()
    p = oracle.params("shadow_sa", est, "window", radius=3, light=light, seed=1)
    gh = occ.hit_u32()
    for t in tiles(case.gb.width, case.gb.height, ntiles, 32, seed=41):
        hr = oracle.halo_region(p, case.gb.width, case.gb.height, t)
        rec = oracle.records(case.osc, case.gb, p, hr)
        res = oracle.reuse(case.osc, case.gb, p, rec, t)
        inside = np.zeros_like(case.gb.valid)
        inside[hr[1]:hr[3], hr[0]:hr[2]] = True
        st = compare_values(gpu, res, region=t, exclude=mismatch_reach(np.where(inside, gh, rec.hit), rec, p))
        log(f"    tile {t}: {st}")


@pytest.mark.parametrize("W,H", [(1, 1), (37, 23), (64, 1)])
def test_small_and_ragged_frames_at_the_largest_window(ocr, W, H):
    # radius 8 stages 6 floats per receiver for the bilinear density (more
    # than 64 KB of LDS per block)
    s = scenes.build([scenes.FLOOR, scenes.plate_y(0.5, -0.5, 0.02, -3, 3)])
    gb = scenes.floor_grid(W, H, 0.02, x0=-0.3, z0=-0.2)
    light = w.RectLight(np.array([0.2, 1.0, 0.1], np.float32), np.array([1.2, 0, 0], np.float32),
                        np.array([0, 0, 1.2], np.float32), 1)
    case = Case(ocr, f"floor_{W}x{H}", s, gb, light)
    occ = _trace(ocr, case, 4)
    for mode in ("shadow", "shadow_sa", "di"):
        for pattern, size, est in [("window", 8, "unbiased"), ("window", 8, "biased"), ("group", 8, "unbiased")]:
            log(f"[bilinear ragged {W}x{H}] {mode} {pattern} {size} {est}")
            gpu = _reuse(ocr, case, mode, occ, ocr.reuse_params(pattern, size, size, est))
            p = oracle.params(mode, est, pattern, radius=size, group_n=size, light=light, seed=4)
            rec, res = oracle.frame(case.osc, gb, p)
            compare_values(gpu, res, exclude=mismatch_reach(occ.hit_u32(), rec, p))
