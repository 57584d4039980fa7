"""Mirror symmetry of the reuse estimators on the GPU: the scene, G-buffer
and occluder records mirrored in x (image columns reversed) give the mirrored
estimate.  The sliding window and the 4-pixel-wide groups of an image whose
width is a multiple of 4 are symmetric, every pair density sees exactly
negated inputs (its products are then exact), and only the order of the box
sums and the validation segments' near-edge decisions differ, so estimates
agree within 1e-4 except at a few grazing segments."""
import numpy as np
import pytest

import workloads as w
from gpu_util import log, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


def _mirror_gbuffer(gb):
    m = w.GBuffer(pos=gb.pos[:, ::-1].copy(), nrm=gb.nrm[:, ::-1].copy(), prim=gb.prim[:, ::-1].copy())
    m.pos[..., 0] *= -1.0
    m.nrm[..., 0] *= -1.0
    return m


def _mirror_records(ocr, occ, H, W):
    m = ocr.Occluders.empty(H, W)
    m.dz.copy_(torch.flip(occ.dz, dims=[1]))
    m.nz.copy_(torch.flip(occ.nz, dims=[1]))
    m.hit.copy_(torch.flip(occ.hit, dims=[1]))
    m.dz[..., 0] *= -1.0
    m.nz[..., 0] *= -1.0
    return m


def _check(a, b, name):
    d = np.abs(a - b[:, ::-1])
    bad = (d > 1e-4).mean()
    log(f"    {name}: max diff {d.max():.2e}, beyond 1e-4: {bad:.5f}")
    assert bad <= 1e-3, (name, bad)


@pytest.mark.parametrize("mode", ["ao", "shadow"])
def test_mirrored_scene_gives_mirrored_estimate(ocr, mode):
    if mode == "ao":
        s = w.boxes_scene(1)
        gb = w.render_gbuffer(s, w.boxes_camera(96, 64))
        R, light = 1.0, None
    else:
        s = w.terrain_scene(2)
        gb = w.render_gbuffer(s, w.terrain_camera(480, 270))
        R, light = 2.0, w.terrain_light()  # centred on x = 0 and symmetric: its own mirror image
    H, W = gb.prim.shape
    Vm = s.V.copy()
    Vm[:, 0] *= -1.0
    bvh, bvh_m = ocr.build_bvh(s.V, s.F), ocr.build_bvh(Vm, s.F)
    dg, dg_m = ocr.DeviceGBuffer.from_host(gb), ocr.DeviceGBuffer.from_host(_mirror_gbuffer(gb))
    occ = ocr.trace_occluders(bvh, dg, mode, R, light, 5, 0)
    torch.cuda.synchronize()
    occ_m = _mirror_records(ocr, occ, H, W)
    for pattern, size, est in [("window", 3, "biased"), ("window", 3, "unbiased"), ("window", 2, "none"),
                               ("group", 8, "biased"), ("group", 8, "unbiased")]:
        p = ocr.reuse_params(pattern, size, size, est)
        if mode == "ao":
            a = to_np(ocr.reuse_ao(bvh, dg, occ, R, p))
            b = to_np(ocr.reuse_ao(bvh_m, dg_m, occ_m, R, p))
        else:
            a = to_np(ocr.reuse_shadow(bvh, dg, occ, light, p))
            b = to_np(ocr.reuse_shadow(bvh_m, dg_m, occ_m, light, p))
        torch.cuda.synchronize()
        _check(a, b, f"{mode} {pattern} {size} {est}")
