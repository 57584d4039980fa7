"""Python binding of the MI355X occlusion-point-reuse library (``libocr.so``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (CUDA tensors on ROCm) and the
current stream; the C-ABI takes raw pointers.  The names mirror ``ocr.h``.
There is no fallback: if the library is missing or the device is not a
gfx950 GPU, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libocr.so")

OCR_AO, OCR_SHADOW = 0, 1
OCR_NOREUSE, OCR_BIASED, OCR_UNBIASED = 0, 1, 2
OCR_WINDOW, OCR_GROUP = 0, 1
HIT_MISS = 0xFFFFFFFF
HIT_SELF = 0xFFFFFFFE

MODES = {"ao": OCR_AO, "shadow": OCR_SHADOW}
# effects of a batched view or a served request: the trace modes plus the
# light effects that reuse shadow records
REQUEST_MODES = dict(MODES, shadow_sa=2, di=3)
ESTIMATORS = {"none": OCR_NOREUSE, "biased": OCR_BIASED, "unbiased": OCR_UNBIASED}
PATTERNS = {"window": OCR_WINDOW, "group": OCR_GROUP}


class OcrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ocr status {status}: {msg}")
        self.status = status


class _GBuffer(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("nrm", ctypes.c_void_p), ("prim", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class _Light(ctypes.Structure):
    _fields_ = [("center", ctypes.c_float * 3), ("edge_u", ctypes.c_float * 3), ("edge_v", ctypes.c_float * 3),
                ("pdf", ctypes.c_int32)]


OCR_LIGHT_UNIFORM, OCR_LIGHT_BILINEAR = 0, 1


class _Occ(ctypes.Structure):
    _fields_ = [("dz", ctypes.c_void_p), ("nz", ctypes.c_void_p), ("hit", ctypes.c_void_p)]


class ReuseParams(ctypes.Structure):
    _fields_ = [("pattern", ctypes.c_int32), ("radius", ctypes.c_int32), ("group_n", ctypes.c_int32),
                ("estimator", ctypes.c_int32), ("dark_guard", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("validated", ctypes.c_int32)]


class BvhInfo(ctypes.Structure):
    _fields_ = [("ntris", ctypes.c_int64), ("nnodes", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("max_leaf", ctypes.c_int32), ("device_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double)]


class ViewDesc(ctypes.Structure):
    _fields_ = [("bvh", ctypes.c_void_p), ("gbuf", _GBuffer), ("mode", ctypes.c_int32), ("ao_radius", ctypes.c_float),
                ("light", _Light), ("seed", ctypes.c_uint64), ("sample", ctypes.c_uint32), ("params", ReuseParams),
                ("out", ctypes.c_void_p), ("radiance", ctypes.c_float), ("albedo", ctypes.c_float)]


OCR_PACK_ROW, OCR_PACK_BLOCK8, OCR_PACK_MORTON = 0, 1, 2
PACKINGS = {"row": OCR_PACK_ROW, "block8": OCR_PACK_BLOCK8, "morton": OCR_PACK_MORTON}


class PlanTuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("packing", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nviews", ctypes.c_int32), ("pixels", ctypes.c_int64), ("trace_items", ctypes.c_int64),
                ("reuse_items", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("tuning", PlanTuning),
                ("tuned", ctypes.c_int32), ("candidates", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("best_trace_ms", ctypes.c_double), ("from_cache", ctypes.c_int32)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("poll_us", ctypes.c_int32), ("mock", ctypes.c_int32), ("mock_ns_per_pixel", ctypes.c_double),
                ("fault_every", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("scene_id", ctypes.c_int32), ("view", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("ao_radius", ctypes.c_float), ("light", _Light), ("seed", ctypes.c_uint64),
                ("sample", ctypes.c_uint32), ("params", ReuseParams), ("out", ctypes.c_void_p),
                ("arrival_ms", ctypes.c_double), ("radiance", ctypes.c_float), ("albedo", ctypes.c_float)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("out", ctypes.c_void_p), ("arrival_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("refused", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int64), ("waited_for_memory", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64), ("max_in_flight", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("frames_per_s", ctypes.c_double), ("failed", ctypes.c_int64)]


EXPORTS = ["ocr_build_bvh", "ocr_build_bvh_host", "ocr_bvh_free", "ocr_bvh_get_info", "ocr_trace_occluders",
           "ocr_trace_occluders_counted", "ocr_sample_rays",
           "ocr_workspace_bytes", "ocr_validate_pairs",
           "ocr_reuse_ao", "ocr_reuse_ao_noalloc", "ocr_reuse_shadow", "ocr_reuse_shadow_solid_angle", "ocr_reuse_direct_illumination",
           "ocr_trace_occluders_lights", "ocr_reuse_shadow_lights", "ocr_validate_pairs_lights",
           "ocr_filter_values",
           "ocr_light_reuse_shadow", "ocr_scale", "ocr_last_error",
           "ocr_version",
           "ocr_plan_create", "ocr_plan_launch", "ocr_plan_get_info", "ocr_plan_get_records", "ocr_plan_free",
           "ocr_server_create", "ocr_server_add_scene", "ocr_server_submit", "ocr_server_poll",
           "ocr_server_release", "ocr_server_drain", "ocr_server_get_stats", "ocr_server_now_ms",
           "ocr_server_destroy"]

_lib = None


def lib():
    """Load libocr.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OcrError(-4, f"{LIB_PATH} is missing: build it first (python -m paper_2607_23122_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.ocr_build_bvh.restype = i32
    L.ocr_build_bvh.argtypes = [vp, i64, vp, i64, vp, ctypes.POINTER(vp)]
    L.ocr_build_bvh_host.restype = i32
    L.ocr_build_bvh_host.argtypes = [vp, i64, vp, i64, vp, i64, vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.ocr_bvh_free.restype = i32
    L.ocr_bvh_free.argtypes = [vp]
    L.ocr_bvh_get_info.restype = i32
    L.ocr_bvh_get_info.argtypes = [vp, ctypes.POINTER(BvhInfo)]
    L.ocr_trace_occluders.restype = i32
    L.ocr_trace_occluders.argtypes = [vp, ctypes.POINTER(_GBuffer), i32, ctypes.c_float, ctypes.POINTER(_Light),
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_Occ), vp]
    L.ocr_trace_occluders_counted.restype = i32
    L.ocr_trace_occluders_counted.argtypes = [vp, ctypes.POINTER(_GBuffer), i32, ctypes.c_float,
                                              ctypes.POINTER(_Light), ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.POINTER(_Occ), vp, vp]
    L.ocr_sample_rays.restype = i32
    L.ocr_sample_rays.argtypes = [ctypes.POINTER(_GBuffer), i32, ctypes.POINTER(_Light), ctypes.c_uint64,
                                  ctypes.c_uint32, vp, vp, vp, vp]
    L.ocr_workspace_bytes.restype = ctypes.c_size_t
    L.ocr_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(ReuseParams)]
    L.ocr_validate_pairs.restype = i32
    L.ocr_validate_pairs.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ), i32, ctypes.c_float,
                                     ctypes.POINTER(_Light), ctypes.POINTER(ReuseParams), vp, ctypes.c_size_t, vp,
                                     vp]
    L.ocr_reuse_ao.restype = i32
    L.ocr_reuse_ao.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ), ctypes.c_float,
                               ctypes.POINTER(ReuseParams), vp, ctypes.c_size_t, vp, vp]
    L.ocr_reuse_ao_noalloc.restype = i32
    L.ocr_reuse_ao_noalloc.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ), ctypes.c_float,
                                       ctypes.POINTER(ReuseParams), vp, vp]
    L.ocr_reuse_shadow.restype = i32
    L.ocr_reuse_shadow.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ), ctypes.POINTER(_Light),
                                   ctypes.POINTER(ReuseParams), vp, ctypes.c_size_t, vp, vp]
    L.ocr_reuse_shadow_solid_angle.restype = i32
    L.ocr_reuse_shadow_solid_angle.argtypes = L.ocr_reuse_shadow.argtypes
    L.ocr_reuse_direct_illumination.restype = i32
    L.ocr_reuse_direct_illumination.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ),
                                                ctypes.POINTER(_Light), ctypes.c_float, ctypes.c_float,
                                                ctypes.POINTER(ReuseParams), vp, ctypes.c_size_t, vp, vp]
    L.ocr_trace_occluders_lights.restype = i32
    L.ocr_trace_occluders_lights.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Light), i32,
                                             ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_Occ), vp]
    L.ocr_reuse_shadow_lights.restype = i32
    L.ocr_reuse_shadow_lights.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ), ctypes.POINTER(_Light),
                                          i32, ctypes.POINTER(ReuseParams), vp, ctypes.c_size_t, vp, vp]
    L.ocr_validate_pairs_lights.restype = i32
    L.ocr_validate_pairs_lights.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Occ),
                                            ctypes.POINTER(_Light), i32, ctypes.POINTER(ReuseParams), vp,
                                            ctypes.c_size_t, vp, vp]
    L.ocr_filter_values.restype = i32
    L.ocr_filter_values.argtypes = [ctypes.POINTER(_GBuffer), ctypes.POINTER(ReuseParams), vp, vp, vp]
    L.ocr_light_reuse_shadow.restype = i32
    L.ocr_light_reuse_shadow.argtypes = [vp, ctypes.POINTER(_GBuffer), ctypes.POINTER(_Light), ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.POINTER(ReuseParams), vp, vp]
    L.ocr_scale.restype = i32
    L.ocr_scale.argtypes = [vp, i64, ctypes.c_float, vp]
    P = ctypes.POINTER
    L.ocr_plan_create.restype = i32
    L.ocr_plan_create.argtypes = [P(ViewDesc), i32, P(PlanTuning), vp, P(vp)]
    L.ocr_plan_launch.restype = i32
    L.ocr_plan_launch.argtypes = [vp, vp]
    L.ocr_plan_get_info.restype = i32
    L.ocr_plan_get_info.argtypes = [vp, P(PlanInfo)]
    L.ocr_plan_get_records.restype = i32
    L.ocr_plan_get_records.argtypes = [vp, i32, P(_Occ)]
    L.ocr_plan_free.restype = i32
    L.ocr_plan_free.argtypes = [vp]
    L.ocr_server_create.restype = i32
    L.ocr_server_create.argtypes = [P(ServerOptions), P(vp)]
    L.ocr_server_add_scene.restype = i32
    L.ocr_server_add_scene.argtypes = [vp, vp, P(_GBuffer), i32, P(i32)]
    L.ocr_server_submit.restype = i32
    L.ocr_server_submit.argtypes = [vp, P(Request), P(ctypes.c_uint64)]
    L.ocr_server_poll.restype = i32
    L.ocr_server_poll.argtypes = [vp, P(Result), i32, P(i32)]
    L.ocr_server_release.restype = i32
    L.ocr_server_release.argtypes = [vp, ctypes.c_uint64]
    L.ocr_server_drain.restype = i32
    L.ocr_server_drain.argtypes = [vp]
    L.ocr_server_get_stats.restype = i32
    L.ocr_server_get_stats.argtypes = [vp, P(ServerStats)]
    L.ocr_server_now_ms.restype = ctypes.c_double
    L.ocr_server_now_ms.argtypes = []
    L.ocr_server_destroy.restype = i32
    L.ocr_server_destroy.argtypes = [vp]
    L.ocr_last_error.restype = ctypes.c_char_p
    L.ocr_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise OcrError(status, lib().ocr_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise OcrError(-1, "expected a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise OcrError(-1, "expected a contiguous tensor")
    return t.data_ptr()


# ---------------------------------------------------------------------------
# Device-side inputs
# ---------------------------------------------------------------------------
@dataclass
class DeviceGBuffer:
    pos: object   # torch.float32 [H,W,3]
    nrm: object   # torch.float32 [H,W,3]
    prim: object  # torch.int32 [H,W] holding uint32 bit patterns

    @property
    def height(self) -> int:
        return int(self.prim.shape[0])

    @property
    def width(self) -> int:
        return int(self.prim.shape[1])

    @classmethod
    def from_host(cls, gb, device="cuda"):
        import torch
        pos = torch.from_numpy(np.ascontiguousarray(gb.pos, np.float32)).to(device)
        nrm = torch.from_numpy(np.ascontiguousarray(gb.nrm, np.float32)).to(device)
        prim = torch.from_numpy(np.ascontiguousarray(gb.prim, np.uint32).view(np.int32)).to(device)
        return cls(pos, nrm, prim)

    def c(self) -> _GBuffer:
        return _GBuffer(_dptr(self.pos), _dptr(self.nrm), _dptr(self.prim), self.width, self.height)


def light_struct(light) -> _Light:
    """A light description: an object with as_array() (centre, e_u, e_v) and
    an optional pdf (OCR_LIGHT_UNIFORM / OCR_LIGHT_BILINEAR), or 9 floats
    (uniform density)."""
    la = light.as_array() if hasattr(light, "as_array") else np.asarray(light, np.float32)
    s = _Light()
    for i in range(3):
        s.center[i] = float(la[i])
        s.edge_u[i] = float(la[3 + i])
        s.edge_v[i] = float(la[6 + i])
    s.pdf = int(getattr(light, "pdf", OCR_LIGHT_UNIFORM))
    return s


def _is_light_list(light) -> bool:
    return isinstance(light, (list, tuple))


def light_array(lights):
    """A C array of light descriptions (shadows of several lights)."""
    arr = (_Light * len(lights))()
    for k, lt in enumerate(lights):
        arr[k] = light_struct(lt)
    return arr


@dataclass
class Occluders:
    dz: object   # torch.float32 [H,W,3]
    nz: object   # torch.float32 [H,W,3]
    hit: object  # torch.int32 [H,W] (uint32 bit patterns)

    @classmethod
    def empty(cls, H, W, device="cuda"):
        import torch
        return cls(torch.zeros((H, W, 3), dtype=torch.float32, device=device),
                   torch.zeros((H, W, 3), dtype=torch.float32, device=device),
                   torch.zeros((H, W), dtype=torch.int32, device=device))

    def c(self) -> _Occ:
        return _Occ(_dptr(self.dz), _dptr(self.nz), _dptr(self.hit))

    def hit_u32(self) -> np.ndarray:
        return self.hit.cpu().numpy().view(np.uint32)


class BVH:
    """Library-owned acceleration structure (ocr_build_bvh / ocr_bvh_free)."""

    def __init__(self, V, F, stream=None):
        V = np.ascontiguousarray(V, np.float32)
        F = np.ascontiguousarray(F, np.uint32)
        h = ctypes.c_void_p()
        _check(lib().ocr_build_bvh(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], _stream(stream),
                                   ctypes.byref(h)))
        self.h = h
        self.ntris = int(F.shape[0])

    def info(self) -> BvhInfo:
        out = BvhInfo()
        _check(lib().ocr_bvh_get_info(self.h, ctypes.byref(out)))
        return out

    def free(self):
        if getattr(self, "h", None) and self.h.value:
            _check(lib().ocr_bvh_free(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


NODE_DTYPE = np.dtype([("lo_x", "<f4", 4), ("hi_x", "<f4", 4), ("lo_y", "<f4", 4), ("hi_y", "<f4", 4),
                       ("lo_z", "<f4", 4), ("hi_z", "<f4", 4), ("child", "<u4", 4), ("pad", "<u4", 4)])


def build_bvh_host(V, F):
    """The hierarchy ocr_build_bvh uploads, built on the host only (no GPU):
    (nodes as a NODE_DTYPE array, leaf-ordered triangles float32[ntris, 3, 4],
    depth)."""
    V = np.ascontiguousarray(V, np.float32)
    F = np.ascontiguousarray(F, np.uint32)
    nn, depth = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().ocr_build_bvh_host(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], None, 0, None,
                                    ctypes.byref(nn), ctypes.byref(depth)))
    nodes = np.zeros(nn.value, NODE_DTYPE)
    tris = np.zeros((F.shape[0], 3, 4), np.float32)
    _check(lib().ocr_build_bvh_host(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], nodes.ctypes.data,
                                    nodes.size, tris.ctypes.data, ctypes.byref(nn), ctypes.byref(depth)))
    return nodes, tris, int(depth.value)


def build_bvh(V, F, stream=None) -> BVH:
    return BVH(V, F, stream)


def reuse_params(pattern="window", radius=2, group_n=8, estimator="biased", dark_guard=True,
                 accumulate=False, validated=False) -> ReuseParams:
    return ReuseParams(PATTERNS[pattern] if isinstance(pattern, str) else int(pattern), int(radius), int(group_n),
                       ESTIMATORS[estimator] if isinstance(estimator, str) else int(estimator),
                       1 if dark_guard else 0, 1 if accumulate else 0, 1 if validated else 0)


def trace_occluders(bvh: BVH, gbuf: DeviceGBuffer, mode="ao", ao_radius=1.0, light=None, seed=1, sample=0,
                    out: Occluders | None = None, stream=None) -> Occluders:
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    out = out or Occluders.empty(gbuf.height, gbuf.width, gbuf.prim.device)
    g = gbuf.c()
    o = out.c()
    if _is_light_list(light):
        # shadows of several lights (ocr_trace_occluders_lights)
        if m != OCR_SHADOW:
            raise ValueError("a list of lights needs mode 'shadow'")
        arr = light_array(light)
        _check(lib().ocr_trace_occluders_lights(bvh.h, ctypes.byref(g), arr, len(light), int(seed), int(sample),
                                                ctypes.byref(o), _stream(stream)))
        return out
    lp = ctypes.byref(light_struct(light)) if light is not None else None
    _check(lib().ocr_trace_occluders(bvh.h, ctypes.byref(g), m, float(ao_radius), lp, int(seed), int(sample),
                                     ctypes.byref(o), _stream(stream)))
    return out


def trace_occluders_counted(bvh: BVH, gbuf: DeviceGBuffer, stats, mode="ao", ao_radius=1.0, light=None, seed=1,
                            sample=0, out: Occluders | None = None, stream=None) -> Occluders:
    """trace_occluders that also adds (rays, node visits, box tests, triangle
    tests, rays) to `stats` (int64 device tensor of 5)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    out = out or Occluders.empty(gbuf.height, gbuf.width, gbuf.prim.device)
    g = gbuf.c()
    o = out.c()
    lp = ctypes.byref(light_struct(light)) if light is not None else None
    _check(lib().ocr_trace_occluders_counted(bvh.h, ctypes.byref(g), m, float(ao_radius), lp, int(seed),
                                             int(sample), ctypes.byref(o), _dptr(stats), _stream(stream)))
    return out


def sample_rays(gbuf: DeviceGBuffer, mode="ao", light=None, seed=1, sample=0, stream=None):
    """(origin, dir, kind) device tensors of the sample step."""
    import torch
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    dev = gbuf.prim.device
    o = torch.empty((gbuf.height, gbuf.width, 3), dtype=torch.float32, device=dev)
    d = torch.empty((gbuf.height, gbuf.width, 3), dtype=torch.float32, device=dev)
    k = torch.empty((gbuf.height, gbuf.width), dtype=torch.uint8, device=dev)
    g = gbuf.c()
    lp = ctypes.byref(light_struct(light)) if light is not None else None
    _check(lib().ocr_sample_rays(ctypes.byref(g), m, lp, int(seed), int(sample), _dptr(o), _dptr(d), _dptr(k),
                                 _stream(stream)))
    return o, d, k


def workspace_bytes(width, height, params: ReuseParams) -> int:
    return int(lib().ocr_workspace_bytes(int(width), int(height), ctypes.byref(params)))


def _workspace(gbuf, params, workspace):
    import torch
    need = workspace_bytes(gbuf.width, gbuf.height, params)
    if need == 0:
        return None, 0
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=gbuf.prim.device)
    return workspace, int(workspace.numel() * workspace.element_size())


def validate_pairs(bvh: BVH, gbuf: DeviceGBuffer, occ: Occluders, mode="ao", ao_radius=1.0, light=None,
                   params: ReuseParams | None = None, workspace=None, stream=None, stats=None):
    """First-hit validation bits of the unbiased estimator into `workspace`;
    `stats` (optional int64 device tensor of 5) accumulates walks, node
    visits, useful box and triangle tests, and segments."""
    params = params or reuse_params(estimator="unbiased")
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    ws, nbytes = _workspace(gbuf, params, workspace)
    g, o = gbuf.c(), occ.c()
    if _is_light_list(light):
        arr = light_array(light)
        _check(lib().ocr_validate_pairs_lights(bvh.h, ctypes.byref(g), ctypes.byref(o), arr, len(light),
                                               ctypes.byref(params), _dptr(ws), nbytes,
                                               _dptr(stats) if stats is not None else None, _stream(stream)))
        return ws
    lp = ctypes.byref(light_struct(light)) if light is not None else None
    _check(lib().ocr_validate_pairs(bvh.h, ctypes.byref(g), ctypes.byref(o), m, float(ao_radius), lp,
                                    ctypes.byref(params), _dptr(ws), nbytes,
                                    _dptr(stats) if stats is not None else None, _stream(stream)))
    return ws


def reuse_ao(bvh: BVH | None, gbuf: DeviceGBuffer, occ: Occluders, ao_radius: float, params: ReuseParams,
             out=None, workspace=None, stream=None):
    import torch
    out = out if out is not None else torch.empty((gbuf.height, gbuf.width), dtype=torch.float32,
                                                  device=gbuf.prim.device)
    ws, nbytes = _workspace(gbuf, params, workspace)
    g, o = gbuf.c(), occ.c()
    _check(lib().ocr_reuse_ao(bvh.h if bvh is not None else None, ctypes.byref(g), ctypes.byref(o), float(ao_radius),
                              ctypes.byref(params), _dptr(ws) if ws is not None else None, nbytes, _dptr(out),
                              _stream(stream)))
    return out


def reuse_ao_noalloc(bvh: BVH | None, gbuf: DeviceGBuffer, occ: Occluders, ao_radius: float, params: ReuseParams,
                     out, stream=None):
    """ocr_reuse_ao_noalloc: reuse_ao with the library's device scratch in
    place of a workspace (the call allocates nothing; `out` is the caller's)."""
    g, o = gbuf.c(), occ.c()
    _check(lib().ocr_reuse_ao_noalloc(bvh.h if bvh is not None else None, ctypes.byref(g), ctypes.byref(o),
                                      float(ao_radius), ctypes.byref(params), _dptr(out), _stream(stream)))
    return out


def reuse_shadow(bvh: BVH | None, gbuf: DeviceGBuffer, occ: Occluders, light, params: ReuseParams, out=None,
                 workspace=None, stream=None):
    import torch
    out = out if out is not None else torch.empty((gbuf.height, gbuf.width), dtype=torch.float32,
                                                  device=gbuf.prim.device)
    ws, nbytes = _workspace(gbuf, params, workspace)
    g, o = gbuf.c(), occ.c()
    if _is_light_list(light):
        # shadows of several lights (ocr_reuse_shadow_lights)
        arr = light_array(light)
        _check(lib().ocr_reuse_shadow_lights(bvh.h if bvh is not None else None, ctypes.byref(g), ctypes.byref(o),
                                             arr, len(light), ctypes.byref(params),
                                             _dptr(ws) if ws is not None else None, nbytes, _dptr(out),
                                             _stream(stream)))
        return out
    ls = light_struct(light)
    _check(lib().ocr_reuse_shadow(bvh.h if bvh is not None else None, ctypes.byref(g), ctypes.byref(o),
                                  ctypes.byref(ls), ctypes.byref(params), _dptr(ws) if ws is not None else None,
                                  nbytes, _dptr(out), _stream(stream)))
    return out


def reuse_shadow_solid_angle(bvh: BVH | None, gbuf: DeviceGBuffer, occ: Occluders, light, params: ReuseParams,
                             out=None, workspace=None, stream=None):
    """Shadows under the solid-angle definition from OCR_SHADOW records
    (ocr_reuse_shadow_solid_angle)."""
    import torch
    out = out if out is not None else torch.empty((gbuf.height, gbuf.width), dtype=torch.float32,
                                                  device=gbuf.prim.device)
    ws, nbytes = _workspace(gbuf, params, workspace)
    g, o = gbuf.c(), occ.c()
    ls = light_struct(light)
    _check(lib().ocr_reuse_shadow_solid_angle(bvh.h if bvh is not None else None, ctypes.byref(g), ctypes.byref(o),
                                              ctypes.byref(ls), ctypes.byref(params),
                                              _dptr(ws) if ws is not None else None, nbytes, _dptr(out),
                                              _stream(stream)))
    return out


def reuse_direct_illumination(bvh: BVH | None, gbuf: DeviceGBuffer, occ: Occluders, light, params: ReuseParams,
                              radiance=1.0, albedo=1.0, out=None, workspace=None, stream=None):
    """Occluder-domain direct illumination of a Lambertian receiver from
    OCR_SHADOW records (ocr_reuse_direct_illumination)."""
    import torch
    out = out if out is not None else torch.empty((gbuf.height, gbuf.width), dtype=torch.float32,
                                                  device=gbuf.prim.device)
    ws, nbytes = _workspace(gbuf, params, workspace)
    g, o = gbuf.c(), occ.c()
    ls = light_struct(light)
    _check(lib().ocr_reuse_direct_illumination(bvh.h if bvh is not None else None, ctypes.byref(g), ctypes.byref(o),
                                               ctypes.byref(ls), float(radiance), float(albedo),
                                               ctypes.byref(params), _dptr(ws) if ws is not None else None, nbytes,
                                               _dptr(out), _stream(stream)))
    return out


def filter_values(gbuf: DeviceGBuffer, params: ReuseParams, inp, out=None, stream=None):
    """Final-value filtering (the paper's Filter (N) / Light (N) baseline):
    the mean of `inp` over each target's set (ocr_filter_values)."""
    import torch
    out = out if out is not None else torch.empty_like(inp)
    g = gbuf.c()
    _check(lib().ocr_filter_values(ctypes.byref(g), ctypes.byref(params), _dptr(inp), _dptr(out),
                                   _stream(stream)))
    return out


def light_reuse_shadow(bvh: BVH, gbuf: DeviceGBuffer, light, seed: int, sample: int, params: ReuseParams, out=None,
                       stream=None):
    """Light-sample reuse with visibility re-evaluation (the paper's Light (NU)
    baseline, ocr_light_reuse_shadow)."""
    import torch
    out = out if out is not None else torch.empty((gbuf.height, gbuf.width), dtype=torch.float32,
                                                  device=gbuf.prim.device)
    g = gbuf.c()
    ls = light_struct(light)
    _check(lib().ocr_light_reuse_shadow(bvh.h, ctypes.byref(g), ctypes.byref(ls), int(seed), int(sample),
                                        ctypes.byref(params), _dptr(out), _stream(stream)))
    return out


def scale(out, s: float, stream=None):
    _check(lib().ocr_scale(_dptr(out), int(out.numel()), float(s), _stream(stream)))
    return out


def render(bvh: BVH, gbuf: DeviceGBuffer, mode="ao", ao_radius=1.0, light=None, seed=1, nsamples=1,
           first_sample=0, params: ReuseParams | None = None, stream=None):
    """Mean over `nsamples` samples of the per-sample estimate (trace, then
    reuse accumulating into one buffer, then one scale); mode "ao", "shadow"
    or "shadow_sa" (shadows under the solid-angle definition)."""
    import torch
    params = params or reuse_params()
    occ = Occluders.empty(gbuf.height, gbuf.width, gbuf.prim.device)
    out = None
    ws = None
    need = workspace_bytes(gbuf.width, gbuf.height, params)
    if need:
        ws = torch.empty(need, dtype=torch.uint8, device=gbuf.prim.device)
    solid_angle = mode == "shadow_sa"
    for s in range(nsamples):
        trace_occluders(bvh, gbuf, "shadow" if solid_angle else mode, ao_radius, light, seed, first_sample + s, occ,
                        stream)
        p = ReuseParams(params.pattern, params.radius, params.group_n, params.estimator, params.dark_guard,
                        0 if s == 0 else 1, 0)
        if mode in ("ao", OCR_AO):
            out = reuse_ao(bvh, gbuf, occ, ao_radius, p, out, ws, stream)
        elif solid_angle:
            out = reuse_shadow_solid_angle(bvh, gbuf, occ, light, p, out, ws, stream)
        else:
            out = reuse_shadow(bvh, gbuf, occ, light, p, out, ws, stream)
    if nsamples > 1:
        scale(out, 1.0 / nsamples, stream)
    return out


def version() -> str:
    return lib().ocr_version().decode()


_hip = None


def device_to_host(ptr: int, shape, dtype) -> np.ndarray:
    """Copy library-owned device memory (plan records, server-held outputs)
    to a new host array with hipMemcpy of the process's HIP runtime (the one
    torch and libocr.so share).  Synchronous; the caller makes sure the
    producing work has finished."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the runtime libocr.so resolves to)
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(shape, dtype)
    if out.nbytes:
        rc = _hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(int(ptr)), out.nbytes, 2)  # device to host
        if rc != 0:
            raise OcrError(-3, f"hipMemcpy failed ({rc})")
    return out


# ---------------------------------------------------------------------------
# Batched schedule (ocr_plan_*)
# ---------------------------------------------------------------------------
def _mode(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def view_desc(bvh: BVH, gbuf: DeviceGBuffer, out, mode="ao", ao_radius=1.0, light=None, seed=1, sample=0,
              params: ReuseParams | None = None, radiance=1.0, albedo=1.0) -> ViewDesc:
    d = ViewDesc()
    d.bvh = bvh.h.value
    d.gbuf = gbuf.c()
    d.mode = REQUEST_MODES[mode] if isinstance(mode, str) else int(mode)
    d.radiance = float(radiance)
    d.albedo = float(albedo)
    d.ao_radius = float(ao_radius)
    if light is not None:
        d.light = light_struct(light)
    d.seed = int(seed)
    d.sample = int(sample)
    d.params = params or reuse_params()
    d.out = _dptr(out)
    return d


def plan_tuning(tile=(16, 16), packing="block8", use_graph=True) -> PlanTuning:
    return PlanTuning(int(tile[0]), int(tile[1]), PACKINGS[packing] if isinstance(packing, str) else int(packing),
                      1 if use_graph else 0)


class Plan:
    """A batched schedule over many views (ocr_plan_*).  The caller keeps the
    BVHs, G-buffers and output tensors alive; `keep` holds references."""

    def __init__(self, views: list, tuning: PlanTuning | None = None, stream=None, keep=None):
        arr = (ViewDesc * len(views))(*views)
        h = ctypes.c_void_p()
        _check(lib().ocr_plan_create(arr, len(views), ctypes.byref(tuning) if tuning is not None else None,
                                     _stream(stream), ctypes.byref(h)))
        self.h = h
        self.keep = keep

    def launch(self, stream=None):
        _check(lib().ocr_plan_launch(self.h, _stream(stream)))

    def info(self) -> PlanInfo:
        out = PlanInfo()
        _check(lib().ocr_plan_get_info(self.h, ctypes.byref(out)))
        return out

    def records(self, v: int) -> _Occ:
        o = _Occ()
        _check(lib().ocr_plan_get_records(self.h, int(v), ctypes.byref(o)))
        return o

    def records_host(self, v: int, H: int, W: int):
        """(dz, nz, hit) of view v copied to host (after the launch finished)."""
        o = self.records(v)
        return (device_to_host(o.dz, (H, W, 3), np.float32), device_to_host(o.nz, (H, W, 3), np.float32),
                device_to_host(o.hit, (H, W), np.uint32))

    def free(self):
        if getattr(self, "h", None) and self.h.value:
            _check(lib().ocr_plan_free(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Served loop (ocr_server_*)
# ---------------------------------------------------------------------------
def server_now_ms() -> float:
    return float(lib().ocr_server_now_ms())


def request(scene_id: int, view: int, mode="ao", ao_radius=1.0, light=None, seed=1, sample=0,
            params: ReuseParams | None = None, out=None, arrival_ms=0.0, radiance=1.0, albedo=1.0) -> Request:
    r = Request()
    r.scene_id = int(scene_id)
    r.view = int(view)
    r.mode = REQUEST_MODES[mode] if isinstance(mode, str) else int(mode)
    r.radiance = float(radiance)
    r.albedo = float(albedo)
    r.ao_radius = float(ao_radius)
    if light is not None:
        r.light = light_struct(light)
    r.seed = int(seed)
    r.sample = int(sample)
    r.params = params or reuse_params()
    r.out = (_dptr(out) if not isinstance(out, int) else out) if out is not None else None
    r.arrival_ms = float(arrival_ms)
    return r


class Server:
    """Served loop (ocr_server_*): resident scenes, HBM-budget admission,
    concurrent slots.  mock=True runs the scheduler without a device;
    fault_every=k makes every k-th admission fail (failure-handling tests)."""

    def __init__(self, budget_bytes: int, slots: int = 8, max_queue: int = 0, poll_us: int = 0,
                 mock: bool = False, mock_ns_per_pixel: float = 0.0, fault_every: int = 0):
        opt = ServerOptions(int(budget_bytes), int(slots), int(max_queue), int(poll_us), 1 if mock else 0,
                            float(mock_ns_per_pixel), int(fault_every))
        h = ctypes.c_void_p()
        _check(lib().ocr_server_create(ctypes.byref(opt), ctypes.byref(h)))
        self.h = h
        self.keep = []

    def add_scene(self, bvh: BVH | None, gbufs: list) -> int:
        arr = (_GBuffer * len(gbufs))(*[g if isinstance(g, _GBuffer) else g.c() for g in gbufs])
        sid = ctypes.c_int32()
        _check(lib().ocr_server_add_scene(self.h, bvh.h if bvh is not None else None, arr, len(gbufs),
                                          ctypes.byref(sid)))
        self.keep.append((bvh, gbufs))
        return int(sid.value)

    def submit(self, req: Request) -> int:
        t = ctypes.c_uint64()
        _check(lib().ocr_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        return int(t.value)

    def try_submit(self, req: Request):
        """(status, ticket): no exception for refusals."""
        t = ctypes.c_uint64()
        st = lib().ocr_server_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        return int(st), int(t.value)

    def poll(self, max_results: int = 256) -> list:
        buf = (Result * max_results)()
        n = ctypes.c_int32()
        _check(lib().ocr_server_poll(self.h, buf, max_results, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def release(self, ticket: int):
        _check(lib().ocr_server_release(self.h, int(ticket)))

    def drain(self):
        _check(lib().ocr_server_drain(self.h))

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib().ocr_server_get_stats(self.h, ctypes.byref(st)))
        return st

    def destroy(self):
        if getattr(self, "h", None) and self.h.value:
            _check(lib().ocr_server_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
