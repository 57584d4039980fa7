"""CPU oracle for occlusion-point reuse -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The GPU library never does, and this
package imports nothing from it: the two share no code.  The arithmetic lives
in ``ocr_oracle.c`` (plain FP64 C, OpenMP over pixels); this module only
marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MISS = 0xFFFFFFFF
SELF = 0xFFFFFFFE


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "ocr_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("estimator", ctypes.c_int32), ("pattern", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("group_n", ctypes.c_int32), ("dark_guard", ctypes.c_int32),
                ("ao_radius", ctypes.c_double), ("light", ctypes.c_float * 9), ("seed", ctypes.c_uint64),
                ("sample", ctypes.c_uint32), ("light_pdf", ctypes.c_int32), ("nlights", ctypes.c_int32),
                ("more_lights", ctypes.c_float * 27)]


MODES = {"ao": 0, "shadow": 1, "shadow_sa": 2, "di": 3}
ESTIMATORS = {"none": 0, "biased": 1, "unbiased": 2, "filter": 3, "light": 4}
PATTERNS = {"window": 0, "group": 1}


def params(mode="ao", estimator="biased", pattern="window", radius=2, group_n=8, dark_guard=True,
           ao_radius=1.0, light=None, seed=1, sample=0) -> Params:
    p = Params()
    p.mode = MODES[mode]
    p.estimator = ESTIMATORS[estimator]
    p.pattern = PATTERNS[pattern]
    p.radius = int(radius)
    p.group_n = int(group_n)
    p.dark_guard = 1 if dark_guard else 0
    p.ao_radius = float(ao_radius)
    if light is not None:
        # one light, or a list of up to 4 (shadows of several lights)
        lights = list(light) if isinstance(light, (list, tuple)) else [light]
        if not 1 <= len(lights) <= 4:
            raise ValueError("1 to 4 lights")
        for k, lt in enumerate(lights):
            la = lt.as_array() if hasattr(lt, "as_array") else np.asarray(lt, np.float32)
            for i in range(9):
                if k == 0:
                    p.light[i] = float(la[i])
                else:
                    p.more_lights[9 * (k - 1) + i] = float(la[i])
        p.nlights = len(lights)
        # the emitter density samples are drawn from (0 uniform, 1 bilinear);
        # the bilinear density is built for one light and estimators 0-2
        pdfs = [int(getattr(lt, "pdf", 0)) for lt in lights]
        if any(pdfs):
            if len(lights) > 1 or mode == "ao" or p.estimator > 2 or pdfs[0] != 1:
                raise ValueError("the bilinear emitter density takes one light and the no-reuse, "
                                 "biased or unbiased estimator")
            p.light_pdf = 1
    p.seed = int(seed)
    p.sample = int(sample)
    return p


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pp = ctypes.POINTER(Params)
    lib.orc_scene_create.restype = vp
    lib.orc_scene_create.argtypes = [vp, i64, vp, i64, i32]
    lib.orc_scene_free.argtypes = [vp]
    lib.orc_scene_grid_cells.restype = i64
    lib.orc_scene_grid_cells.argtypes = [vp]
    lib.orc_closest.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.orc_any.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_samples.argtypes = [i32, i32, vp, vp, vp, pp, i32, i32, i32, i32, vp, vp, vp]
    lib.orc_records.argtypes = [vp, i32, i32, vp, vp, vp, pp, i32, i32, i32, i32, vp, vp, vp, vp]
    lib.orc_reuse.argtypes = [vp, i32, i32, vp, vp, vp, pp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp]
    lib.orc_render.argtypes = [vp, i32, i32, vp, vp, vp, pp, i32, i32, i32, i32, i32, vp, vp]
    lib.orc_density_ao.restype = f64
    lib.orc_density_ao.argtypes = [vp, vp, vp, vp, f64]
    lib.orc_density_shadow.restype = f64
    lib.orc_density_shadow.argtypes = [vp, vp, vp, vp, vp]
    lib.orc_front_fraction.restype = f64
    lib.orc_front_fraction.argtypes = [vp, vp, vp]
    lib.orc_ao_quadrature.restype = f64
    lib.orc_ao_quadrature.argtypes = [vp, vp, vp, f64, ctypes.c_uint32, i32]
    lib.orc_shadow_quadrature.restype = f64
    lib.orc_shadow_quadrature.argtypes = [vp, vp, vp, vp, ctypes.c_uint32, i32]
    lib.orc_shadow_sa_quadrature.restype = f64
    lib.orc_shadow_sa_quadrature.argtypes = [vp, vp, vp, vp, ctypes.c_uint32, i32]
    lib.orc_solid_angles.argtypes = [vp, vp, vp, vp]
    lib.orc_emitter_irradiance.restype = f64
    lib.orc_emitter_irradiance.argtypes = [vp, vp, vp]
    lib.orc_di_factor.restype = f64
    lib.orc_di_factor.argtypes = [vp, vp, vp, vp]
    lib.orc_di_quadrature.restype = f64
    lib.orc_di_quadrature.argtypes = [vp, vp, vp, vp, ctypes.c_uint32, i32]
    lib.orc_sa_factor.restype = f64
    lib.orc_sa_factor.argtypes = [vp, vp, vp, vp]
    lib.orc_light_q.restype = f64
    lib.orc_light_q.argtypes = [vp, vp, f64, f64]
    lib.orc_pcg4d_first.restype = ctypes.c_uint32
    lib.orc_pcg4d_first.argtypes = [ctypes.c_uint32] * 4 + [vp]
    lib.orc_num_threads.restype = i32
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def pcg4d(a, b, c, d) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    _load().orc_pcg4d_first(a & 0xFFFFFFFF, b & 0xFFFFFFFF, c & 0xFFFFFFFF, d & 0xFFFFFFFF, _ptr(out))
    return out


class Scene:
    """FP64 copy of a triangle scene, brute force or uniform-grid candidates."""

    def __init__(self, V, F, grid: bool = True):
        lib = _load()
        self.V = np.ascontiguousarray(V, np.float32)
        self.F = np.ascontiguousarray(F, np.uint32)
        self.h = lib.orc_scene_create(_ptr(self.V), self.V.shape[0], _ptr(self.F), self.F.shape[0],
                                      1 if grid else 0)
        self.grid = grid

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _load().orc_scene_free(self.h)
                self.h = None
        except Exception:
            pass

    def closest(self, o, d, tmax, inclusive=True, ign0=None, ign1=None):
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        n = o.shape[0]
        tm = np.ascontiguousarray(np.broadcast_to(np.asarray(tmax, np.float64), (n,)))
        i0 = np.full(n, MISS, np.uint32) if ign0 is None else np.ascontiguousarray(np.broadcast_to(ign0, (n,)), np.uint32)
        i1 = np.full(n, MISS, np.uint32) if ign1 is None else np.ascontiguousarray(np.broadcast_to(ign1, (n,)), np.uint32)
        tri = np.zeros(n, np.uint32)
        t = np.zeros(n, np.float64)
        g = np.zeros(n, np.uint8)
        _load().orc_closest(self.h, n, _ptr(o), _ptr(d), _ptr(tm), 1 if inclusive else 0, _ptr(i0), _ptr(i1),
                            _ptr(tri), _ptr(t), _ptr(g))
        return tri, t, g.astype(bool)

    def any_hit(self, o, d, tmax, ign0=None, ign1=None):
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        n = o.shape[0]
        tm = np.ascontiguousarray(np.broadcast_to(np.asarray(tmax, np.float64), (n,)))
        i0 = np.full(n, MISS, np.uint32) if ign0 is None else np.ascontiguousarray(np.broadcast_to(ign0, (n,)), np.uint32)
        i1 = np.full(n, MISS, np.uint32) if ign1 is None else np.ascontiguousarray(np.broadcast_to(ign1, (n,)), np.uint32)
        b = np.zeros(n, np.uint8)
        g = np.zeros(n, np.uint8)
        _load().orc_any(self.h, n, _ptr(o), _ptr(d), _ptr(tm), _ptr(i0), _ptr(i1), _ptr(b), _ptr(g))
        return b.astype(bool), g.astype(bool)

    def ao_quadrature(self, o, n, R, ign=MISS, nstrata=512):
        o = np.ascontiguousarray(o, np.float64)
        n = np.ascontiguousarray(n, np.float64)
        return float(_load().orc_ao_quadrature(self.h, _ptr(o), _ptr(n), float(R), int(ign), int(nstrata)))

    def shadow_quadrature(self, o, n, light, ign=MISS, ngrid=512):
        o = np.ascontiguousarray(o, np.float64)
        n = np.ascontiguousarray(n, np.float64)
        la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
        return float(_load().orc_shadow_quadrature(self.h, _ptr(o), _ptr(n), _ptr(la), int(ign), int(ngrid)))

    def di_quadrature(self, o, n, light, ign=MISS, ngrid=512):
        """Visible irradiance of the unit-radiance light (direct illumination
        in units of rho L_e / pi)."""
        o = np.ascontiguousarray(o, np.float64)
        n = np.ascontiguousarray(n, np.float64)
        la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
        return float(_load().orc_di_quadrature(self.h, _ptr(o), _ptr(n), _ptr(la), int(ign), int(ngrid)))

    def shadow_sa_quadrature(self, o, n, light, ign=MISS, ngrid=512):
        o = np.ascontiguousarray(o, np.float64)
        n = np.ascontiguousarray(n, np.float64)
        la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
        return float(_load().orc_shadow_sa_quadrature(self.h, _ptr(o), _ptr(n), _ptr(la), int(ign), int(ngrid)))


def _gb(gb):
    pos = np.ascontiguousarray(gb.pos, np.float32)
    nrm = np.ascontiguousarray(gb.nrm, np.float32)
    prim = np.ascontiguousarray(gb.prim, np.uint32)
    return pos, nrm, prim


def samples(gb, p: Params, region=None):
    pos, nrm, prim = _gb(gb)
    H, W = prim.shape
    x0, y0, x1, y1 = region if region is not None else (0, 0, W, H)
    o = np.zeros((H, W, 3), np.float32)
    d = np.zeros((H, W, 3), np.float32)
    k = np.full((H, W), 2, np.uint8)
    _load().orc_samples(W, H, _ptr(pos), _ptr(nrm), _ptr(prim), ctypes.byref(p), x0, y0, x1, y1, _ptr(o),
                        _ptr(d), _ptr(k))
    return o, d, k


class Records:
    def __init__(self, H, W):
        self.hit = np.full((H, W), MISS, np.uint32)
        self.z = np.zeros((H, W, 3), np.float64)
        self.nz = np.zeros((H, W, 3), np.float64)
        self.graze = np.zeros((H, W), np.uint8)


def halo_region(p: Params, W, H, region):
    """Pixels whose records the targets of `region` read."""
    x0, y0, x1, y1 = region
    if p.estimator == 0:
        r = [x0, y0, x1, y1]
    elif p.pattern == 0:
        r = [x0 - p.radius, y0 - p.radius, x1 + p.radius, y1 + p.radius]
    else:
        gw = 4 if p.group_n == 8 else (2 if p.group_n >= 2 else 1)
        gh = 2 if p.group_n >= 4 else 1
        r = [(x0 // gw) * gw, (y0 // gh) * gh, -(-x1 // gw) * gw, -(-y1 // gh) * gh]
    return max(r[0], 0), max(r[1], 0), min(r[2], W), min(r[3], H)


def records(scene: Scene, gb, p: Params, region=None, rec: Records | None = None) -> Records:
    pos, nrm, prim = _gb(gb)
    H, W = prim.shape
    x0, y0, x1, y1 = region if region is not None else (0, 0, W, H)
    rec = rec or Records(H, W)
    _load().orc_records(scene.h, W, H, _ptr(pos), _ptr(nrm), _ptr(prim), ctypes.byref(p), x0, y0, x1, y1,
                        _ptr(rec.hit), _ptr(rec.z), _ptr(rec.nz), _ptr(rec.graze))
    return rec


class ReuseResult:
    def __init__(self, H, W):
        self.value = np.zeros((H, W), np.float64)
        self.nvar = np.zeros((H, W), np.uint8)
        self.var = np.zeros((H, W, 8), np.float64)


def reuse(scene: Scene, gb, p: Params, rec: Records, region=None) -> ReuseResult:
    pos, nrm, prim = _gb(gb)
    H, W = prim.shape
    x0, y0, x1, y1 = region if region is not None else (0, 0, W, H)
    out = ReuseResult(H, W)
    _load().orc_reuse(scene.h, W, H, _ptr(pos), _ptr(nrm), _ptr(prim), ctypes.byref(p), _ptr(rec.hit),
                      _ptr(rec.z), _ptr(rec.nz), _ptr(rec.graze), x0, y0, x1, y1, _ptr(out.value),
                      _ptr(out.nvar), _ptr(out.var))
    return out


def frame(scene: Scene, gb, p: Params, region=None):
    """Records over the region's halo, then the estimate over the region."""
    H, W = gb.prim.shape
    region = region if region is not None else (0, 0, W, H)
    rec = records(scene, gb, p, halo_region(p, W, H, region))
    return rec, reuse(scene, gb, p, rec, region)


def render(scene: Scene, gb, p: Params, nsamples: int, region=None):
    """Sum and sum of squares over samples p.sample .. p.sample+nsamples-1."""
    pos, nrm, prim = _gb(gb)
    H, W = prim.shape
    x0, y0, x1, y1 = region if region is not None else (0, 0, W, H)
    s = np.zeros((H, W), np.float64)
    s2 = np.zeros((H, W), np.float64)
    _load().orc_render(scene.h, W, H, _ptr(pos), _ptr(nrm), _ptr(prim), ctypes.byref(p), int(nsamples), x0, y0,
                       x1, y1, _ptr(s), _ptr(s2))
    return s, s2


def density_ao(o, n, z, nz, R) -> float:
    a = [np.ascontiguousarray(v, np.float64) for v in (o, n, z, nz)]
    return float(_load().orc_density_ao(*[_ptr(v) for v in a], float(R)))


def density_shadow(o, n, z, nz, light) -> float:
    a = [np.ascontiguousarray(v, np.float64) for v in (o, n, z, nz)]
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    return float(_load().orc_density_shadow(*[_ptr(v) for v in a], _ptr(la)))


def front_fraction(o, n, light) -> float:
    o = np.ascontiguousarray(o, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    return float(_load().orc_front_fraction(_ptr(o), _ptr(n), _ptr(la)))


def solid_angles(o, n, light):
    """(Omega_A, Omega_front): the light's solid angle at o and its part in
    front of the tangent plane of (o, n)."""
    o = np.ascontiguousarray(o, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    out = np.zeros(2, np.float64)
    _load().orc_solid_angles(_ptr(o), _ptr(n), _ptr(la), _ptr(out))
    return float(out[0]), float(out[1])


def sa_factor(o, n, z, light) -> float:
    a = [np.ascontiguousarray(v, np.float64) for v in (o, n, z)]
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    return float(_load().orc_sa_factor(*[_ptr(v) for v in a], _ptr(la)))


def light_q(o, light, a, b) -> float:
    """Area p_A(y | x) of the bilinear emitter density of receiver point o at
    light coordinates (a, b) of y (|a|, |b| <= 1/2)."""
    oa = np.ascontiguousarray(o, np.float64)
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    return float(_load().orc_light_q(_ptr(oa), _ptr(la), float(a), float(b)))


def emitter_irradiance(o, n, light) -> float:
    a = [np.ascontiguousarray(v, np.float64) for v in (o, n)]
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    return float(_load().orc_emitter_irradiance(*[_ptr(v) for v in a], _ptr(la)))


def di_factor(o, n, z, light) -> float:
    a = [np.ascontiguousarray(v, np.float64) for v in (o, n, z)]
    la = np.ascontiguousarray(light.as_array() if hasattr(light, "as_array") else light, np.float64)
    return float(_load().orc_di_factor(*[_ptr(v) for v in a], _ptr(la)))
