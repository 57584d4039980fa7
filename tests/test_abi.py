"""The C-ABI library loads and exports every entry point include/ocr.h
declares; argument validation rejects bad inputs before touching a device.
(No compute calls: these run without a GPU.)"""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ocr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ocr_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2607_23122_amd as ocr
    lib = ocr.lib()
    names = _declared()
    assert len(names) >= 11, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(ocr.EXPORTS) <= set(names)
    assert "gfx950" in ocr.version()


def test_workspace_bytes():
    import paper_2607_23122_amd as ocr
    assert ocr.workspace_bytes(1920, 1080, ocr.reuse_params("window", 3, 0, "biased")) == 0
    # 13 x 13 pairs per receiver -> 169 bits -> 6 words
    # plus the window validation's per-XCD candidate lists (8 padded counters + 8 x ceil(tiles/8) x 256 slots)
    tiles = 120 * 68
    assert ocr.workspace_bytes(1920, 1080, ocr.reuse_params("window", 3, 0, "unbiased")) == \
        1920 * 1080 * 6 * 4 + (8 * 32 + ((tiles + 7) // 8) * 8 * 256) * 4
    # 4 x 2 groups: offsets in [-3, 3]^2 -> 49 bits -> 2 words, and the same lists
    t2 = 7 * 1
    assert ocr.workspace_bytes(100, 10, ocr.reuse_params("group", 0, 8, "unbiased")) == \
        100 * 10 * 2 * 4 + (8 * 32 + ((t2 + 7) // 8) * 8 * 256) * 4
    assert ocr.workspace_bytes(100, 10, ocr.reuse_params("window", 9, 0, "unbiased")) == 0
    assert ocr.workspace_bytes(0, 10, ocr.reuse_params("window", 3, 0, "unbiased")) == 0


def test_argument_validation_without_device():
    import paper_2607_23122_amd as ocr
    lib = ocr.lib()
    h = ctypes.c_void_p()
    V = np.zeros((3, 3), np.float32)
    F = np.array([[0, 1, 5]], np.uint32)  # vertex 5 out of range
    assert lib.ocr_build_bvh(V.ctypes.data, 3, F.ctypes.data, 1, None, ctypes.byref(h)) == -1
    assert b"references vertex" in lib.ocr_last_error()
    assert lib.ocr_build_bvh(None, 3, F.ctypes.data, 1, None, ctypes.byref(h)) == -1
    assert lib.ocr_build_bvh(V.ctypes.data, 3, F.ctypes.data, 0, None, ctypes.byref(h)) == -1
    Vn = np.array([[0, 0, 0], [1, 0, 0], [np.nan, 1, 0]], np.float32)
    F0 = np.array([[0, 1, 2]], np.uint32)
    assert lib.ocr_build_bvh(Vn.ctypes.data, 3, F0.ctypes.data, 1, None, ctypes.byref(h)) == -1
    # NULL gbuffer / bvh / params
    assert lib.ocr_trace_occluders(None, None, 0, 1.0, None, 1, 0, None, None) == -1
    g = ocr._GBuffer(0, 0, 0, 4, 4)
    assert lib.ocr_reuse_ao(None, ctypes.byref(g), None, 1.0, None, None, 0, None, None) == -1
    assert b"NULL" in lib.ocr_last_error()
    g2 = ocr._GBuffer(8, 8, 8, 0, 4)  # zero width (pointers never dereferenced)
    p = ocr.reuse_params("window", 3, 0, "biased")
    o = ocr._Occ(8, 8, 8)
    assert lib.ocr_reuse_ao(None, ctypes.byref(g2), ctypes.byref(o), 1.0, ctypes.byref(p), None, 0, 8, None) == -1
    g3 = ocr._GBuffer(8, 8, 8, 4, 4)
    assert lib.ocr_reuse_ao(None, ctypes.byref(g3), ctypes.byref(o), float("inf"), ctypes.byref(p), None, 0, 8,
                            None) == -1
    bad = ocr.reuse_params("group", 0, 3, "biased")
    assert lib.ocr_reuse_ao(None, ctypes.byref(g3), ctypes.byref(o), 1.0, ctypes.byref(bad), None, 0, 8, None) == -1
    assert b"group size" in lib.ocr_last_error()
    unb = ocr.reuse_params("window", 3, 0, "unbiased")
    assert lib.ocr_reuse_ao(None, ctypes.byref(g3), ctypes.byref(o), 1.0, ctypes.byref(unb), None, 0, 8, None) == -1
    assert b"workspace" in lib.ocr_last_error()
    # degenerate light
    L = ocr._Light()
    for i in range(3):
        L.edge_u[i] = 0.0
    assert lib.ocr_reuse_shadow(None, ctypes.byref(g3), ctypes.byref(o), ctypes.byref(L), ctypes.byref(p), None, 0,
                                8, None) == -1
    assert b"zero length" in lib.ocr_last_error()
    assert lib.ocr_scale(None, 4, 1.0, None) == -1


def test_noalloc_size_limit_without_device():
    # a frame whose unbiased workspace exceeds the library's 64 MiB scratch is
    # refused before any device call (the pointers are never dereferenced)
    import paper_2607_23122_amd as ocr
    lib = ocr.lib()
    g = ocr._GBuffer(8, 8, 8, 4096, 4096)
    o = ocr._Occ(8, 8, 8)
    p = ocr.reuse_params("window", 3, 0, "unbiased")
    assert ocr.workspace_bytes(4096, 4096, p) > 64 << 20
    assert lib.ocr_reuse_ao_noalloc(None, ctypes.byref(g), ctypes.byref(o), 1.0, ctypes.byref(p), 8, None) == -1
    assert b"scratch" in lib.ocr_last_error()
