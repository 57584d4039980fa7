"""The entry point that allocates nothing (ocr_reuse_ao_noalloc), through
the C-ABI, against ocr_reuse_ao with a caller workspace: the same kernels,
so the same bits, on two calls in a row, the second with a smaller frame
(the device scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

import workloads as w
from gpu_util import log

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


def _frame(ocr, W, H):
    s = w.terrain_scene(2)
    gb = w.render_gbuffer(s, w.terrain_camera(W, H))
    return ocr.build_bvh(s.V, s.F), ocr.DeviceGBuffer.from_host(gb)


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_point(ocr):
    configs = [("window", 3, "unbiased"), ("window", 1, "unbiased"), ("group", 8, "unbiased"), ("window", 3, "biased")]
    for W, H in [(1920, 1080), (480, 270)]:
        bvh, dg = _frame(ocr, W, H)
        occ = ocr.trace_occluders(bvh, dg, "ao", 2.0, None, seed=3, sample=1)
        for pattern, size, est in configs:
            log(f"[noalloc] {W}x{H} {pattern} {size} {est}")
            p = ocr.reuse_params(pattern, size, size, est)
            ref = ocr.reuse_ao(bvh, dg, occ, 2.0, p)
            out = torch.full((H, W), float("nan"), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            g, o = dg.c(), occ.c()
            st = ocr.lib().ocr_reuse_ao_noalloc(bvh.h, ctypes.byref(g), ctypes.byref(o), 2.0, ctypes.byref(p),
                                                out.data_ptr(), ocr._stream(None))
            assert st == 0, ocr.lib().ocr_last_error()
            torch.cuda.synchronize()
            a, b = out.cpu().numpy(), ref.cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        bvh.free()


@pytest.mark.gpu
def test_noalloc_refuses_what_it_cannot_hold(ocr):
    s = w.boxes_scene(1)
    gb = w.render_gbuffer(s, w.boxes_camera(64, 64))
    bvh = ocr.build_bvh(s.V, s.F)
    dg = ocr.DeviceGBuffer.from_host(gb)
    occ = ocr.trace_occluders(bvh, dg, "ao", 1.0, None, seed=1)
    out = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    # validated bits are not taken: the validation runs within the call
    p = ocr.reuse_params("window", 2, 0, "unbiased", validated=True)
    with pytest.raises(ocr.OcrError) as e:
        ocr.reuse_ao_noalloc(bvh, dg, occ, 1.0, p, out)
    assert e.value.status == -1
    torch.cuda.synchronize()
