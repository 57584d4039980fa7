"""Seeded synthetic workloads: scenes, cameras, lights and G-buffers.

This module only makes inputs.  It holds none of the method's arithmetic
(no sampling, no occluder tracing, no densities, no reuse): the oracle and
the GPU library both consume what it produces and neither is called from it.

The paper evaluates on Falcor scenes that are not available here and whose
sizes it does not state (Sec. 6, AO and shadow scene lists); these generators
stand in for them with scenes of the same kind -- a ground with boxes, and a
displaced terrain with spheres -- rendered at the paper's resolution (1080p,
Sec. 6 experimental setup) with one sample per pixel.

Conventions: y is up, units are metres, triangles are indexed in generation
order, the pinhole camera has a 60 degree vertical field of view, pixel
centres at (px+1/2, py+1/2) and row 0 at the top.  Scene randomness comes
from numpy's PCG64 stream seeded per scene.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgbuf.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the FP64 G-buffer writer with gcc (OpenMP)."""
    src = os.path.join(_HERE, "_gbuf.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
                               "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.gb_render.restype = ctypes.c_int
        lib.gb_render.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


# --------------------------------------------------------------------------
# Data holders
# --------------------------------------------------------------------------
@dataclass
class Scene:
    V: np.ndarray  # float32 [nv,3]
    F: np.ndarray  # uint32 [nt,3]
    name: str = ""

    @property
    def ntris(self) -> int:
        return int(self.F.shape[0])


@dataclass
class Camera:
    eye: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    tan_half: float
    width: int
    height: int


@dataclass
class GBuffer:
    pos: np.ndarray   # float32 [H,W,3]
    nrm: np.ndarray   # float32 [H,W,3]
    prim: np.ndarray  # uint32 [H,W], 0xFFFFFFFF = background

    @property
    def height(self) -> int:
        return int(self.prim.shape[0])

    @property
    def width(self) -> int:
        return int(self.prim.shape[1])

    @property
    def valid(self) -> np.ndarray:
        return self.prim != 0xFFFFFFFF


@dataclass
class RectLight:
    """Rectangle centre c and edge vectors e_u, e_v; the emitting side is
    normalize(e_u x e_v).  pdf: the density its samples are drawn from, 0
    uniform over the area, 1 the receiver-dependent bilinear density."""
    center: np.ndarray
    edge_u: np.ndarray
    edge_v: np.ndarray
    pdf: int = 0

    def as_array(self) -> np.ndarray:
        return np.concatenate([self.center, self.edge_u, self.edge_v]).astype(np.float32)


# --------------------------------------------------------------------------
# Geometry builders
# --------------------------------------------------------------------------
def _box(lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    V = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], dtype=np.float64)
    F = np.array([[0, 2, 1], [0, 3, 2],  # z0 face
                  [4, 5, 6], [4, 6, 7],  # z1 face
                  [0, 1, 5], [0, 5, 4],  # y0 face
                  [3, 6, 2], [3, 7, 6],  # y1 face
                  [0, 4, 7], [0, 7, 3],  # x0 face
                  [1, 2, 6], [1, 6, 5]], dtype=np.int64)  # x1 face
    return V, F


def _merge(parts):
    Vs, Fs, off = [], [], 0
    for V, F in parts:
        Vs.append(V)
        Fs.append(F + off)
        off += V.shape[0]
    return np.concatenate(Vs).astype(np.float32), np.concatenate(Fs).astype(np.uint32)


def quad(corner, eu, ev):
    """Two triangles spanning corner, corner+eu, corner+eu+ev, corner+ev."""
    c = np.asarray(corner, np.float64)
    eu = np.asarray(eu, np.float64)
    ev = np.asarray(ev, np.float64)
    V = np.stack([c, c + eu, c + eu + ev, c + ev])
    F = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64)
    return V, F


def boxes_scene(seed: int = 1, nboxes: int = 64, half: float = 10.0) -> Scene:
    """Ground quad [-half,half]^2 at y=0 (2 triangles) plus axis-aligned boxes
    with sizes U[0.2,2]^3 resting on the ground, centres uniform in the quad
    (12 triangles each): 770 triangles for 64 boxes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [quad((-half, 0.0, -half), (2 * half, 0, 0), (0, 0, 2 * half))]
    for _ in range(nboxes):
        s = rng.uniform(0.2, 2.0, size=3)
        cx, cz = rng.uniform(-half, half, size=2)
        lo = (cx - s[0] / 2, 0.0, cz - s[2] / 2)
        hi = (cx + s[0] / 2, s[1], cz + s[2] / 2)
        parts.append(_box(lo, hi))
    V, F = _merge(parts)
    return Scene(V, F, name=f"boxes(seed={seed},n={nboxes})")


def _icosphere(level: int = 2):
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}
        nF = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nF += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nF
    return np.array(V), np.array(F, dtype=np.int64)


_ICO2 = None


def icosphere2():
    """Level-2 icosphere: 162 vertices, 320 triangles, unit radius."""
    global _ICO2
    if _ICO2 is None:
        _ICO2 = _icosphere(2)
    return _ICO2


def _hash2(ix: np.ndarray, iz: np.ndarray, octave: int, seed: int) -> np.ndarray:
    """Integer lattice hash (PCG-style multiply/xorshift) -> value in [-1,1]."""
    with np.errstate(over="ignore"):
        h = (ix.astype(np.uint32) * np.uint32(0x8DA6B343)) ^ (iz.astype(np.uint32) * np.uint32(0xD8163841))
        h = h ^ np.uint32((octave * 0x9E3779B9 + seed * 0x85EBCA6B) & 0xFFFFFFFF)
        h = h * np.uint32(747796405) + np.uint32(2891336453)
        h = ((h >> ((h >> np.uint32(28)) + np.uint32(4))) ^ h) * np.uint32(277803737)
        h = (h >> np.uint32(22)) ^ h
    return (h.astype(np.float64) / 4294967295.0) * 2.0 - 1.0


def fbm(x: np.ndarray, z: np.ndarray, seed: int, octaves: int = 6, wavelength: float = 50.0,
        lacunarity: float = 2.0, gain: float = 0.5) -> np.ndarray:
    """fBm of hashed 2D value noise with quintic interpolation (unnormalised)."""
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64)
    out = np.zeros(np.broadcast(x, z).shape)
    amp, lam = 1.0, wavelength
    for o in range(octaves):
        gx, gz = x / lam, z / lam
        ix, iz = np.floor(gx), np.floor(gz)
        fx, fz = gx - ix, gz - iz
        ux = fx * fx * fx * (fx * (fx * 6 - 15) + 10)
        uz = fz * fz * fz * (fz * (fz * 6 - 15) + 10)
        ixi, izi = ix.astype(np.int64), iz.astype(np.int64)
        v00 = _hash2(ixi, izi, o, seed)
        v10 = _hash2(ixi + 1, izi, o, seed)
        v01 = _hash2(ixi, izi + 1, o, seed)
        v11 = _hash2(ixi + 1, izi + 1, o, seed)
        a = v00 + (v10 - v00) * ux
        b = v01 + (v11 - v01) * ux
        out += amp * (a + (b - a) * uz)
        amp *= gain
        lam /= lacunarity
    return out


def terrain_scene(seed: int = 2, cells: int = 512, nspheres: int = 2000, half: float = 100.0,
                  sphere_half: float = 60.0, hmax: float = 4.0) -> Scene:
    """Displaced terrain over [-half,half]^2 as cells x cells quads (fixed
    diagonal split, 2*cells^2 triangles), heights = fBm normalised to
    [-hmax,hmax], plus level-2 icospheres (320 triangles each) with radius
    U[0.1,1.5] at centres (x,z) ~ U[-sphere_half,sphere_half]^2 and
    y = h(x,z) + r U[-0.25,0.75]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cells + 1
    g = np.linspace(-half, half, n)
    X, Z = np.meshgrid(g, g, indexing="xy")  # X[iz, ix]
    Hraw = fbm(X, Z, seed)
    lo, hi = Hraw.min(), Hraw.max()

    def height(x, z):
        return -hmax + 2 * hmax * (fbm(x, z, seed) - lo) / (hi - lo)

    Hn = -hmax + 2 * hmax * (Hraw - lo) / (hi - lo)
    Vt = np.stack([X.ravel(), Hn.ravel(), Z.ravel()], axis=1)
    iz, ix = np.meshgrid(np.arange(cells), np.arange(cells), indexing="ij")
    v00 = (iz * n + ix).ravel()
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    Ft = np.empty((2 * cells * cells, 3), np.int64)
    Ft[0::2] = np.stack([v00, v01, v11], axis=1)
    Ft[1::2] = np.stack([v00, v11, v10], axis=1)
    parts = [(Vt, Ft)]
    if nspheres > 0:
        Vs, Fs = icosphere2()
        r = rng.uniform(0.1, 1.5, size=nspheres)
        cxz = rng.uniform(-sphere_half, sphere_half, size=(nspheres, 2))
        dy = rng.uniform(-0.25, 0.75, size=nspheres)
        cy = height(cxz[:, 0], cxz[:, 1]) + r * dy
        centres = np.stack([cxz[:, 0], cy, cxz[:, 1]], axis=1)
        allV = (Vs[None, :, :] * r[:, None, None] + centres[:, None, :]).reshape(-1, 3)
        offs = (np.arange(nspheres) * Vs.shape[0])[:, None, None]
        allF = (Fs[None, :, :] + offs).reshape(-1, 3)
        parts.append((allV, allF))
    V, F = _merge(parts)
    return Scene(V, F, name=f"terrain(seed={seed},cells={cells},spheres={nspheres})")


# --------------------------------------------------------------------------
# Camera, light, G-buffer
# --------------------------------------------------------------------------
def pinhole(eye, look_at, width: int, height: int, vfov_deg: float = 60.0) -> Camera:
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(look_at, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    world_up = np.array([0.0, 1.0, 0.0])
    right = np.cross(world_up, fwd)
    right /= np.linalg.norm(right)
    up = np.cross(fwd, right)
    return Camera(eye, fwd, right, up, float(np.tan(np.radians(vfov_deg) / 2)), int(width), int(height))


def orbit_camera(v: int, nviews: int, width: int, height: int, eye=(0.0, 45.0, -30.0),
                 look_at=(0.0, 0.0, 12.0)) -> Camera:
    """Camera at the height and horizontal distance of `eye` from `look_at`,
    rotated by 2*pi*v/nviews about the vertical axis through `look_at`."""
    eye = np.asarray(eye, np.float64)
    la = np.asarray(look_at, np.float64)
    off = eye - la
    phi = 2.0 * np.pi * v / nviews
    c, s = np.cos(phi), np.sin(phi)
    rot = np.array([off[0] * c + off[2] * s, off[1], -off[0] * s + off[2] * c])
    return pinhole(la + rot, la, width, height)


def render_gbuffer(scene: Scene, cam: Camera) -> GBuffer:
    lib = _load()
    W, H = cam.width, cam.height
    pos = np.zeros((H, W, 3), np.float32)
    nrm = np.zeros((H, W, 3), np.float32)
    prim = np.zeros((H, W), np.uint32)
    V = np.ascontiguousarray(scene.V, np.float32)
    F = np.ascontiguousarray(scene.F, np.uint32)
    vecs = [np.ascontiguousarray(a, np.float64) for a in (cam.eye, cam.fwd, cam.right, cam.up)]
    rc = lib.gb_render(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0],
                       *[a.ctypes.data for a in vecs], cam.tan_half, W, H,
                       pos.ctypes.data, nrm.ctypes.data, prim.ctypes.data)
    if rc != 0:
        raise RuntimeError("gb_render failed")
    return GBuffer(pos, nrm, prim)


def plane_gbuffer(width: int, height: int, spacing: float, origin=(0.0, 0.0, 0.0), prim: int = 0,
                  normal=(0.0, 1.0, 0.0)) -> GBuffer:
    """Receivers on a regular grid in the y=origin[1] plane (x along columns,
    z along rows), all sharing one primitive id and normal.  Used for small
    hand-built test configurations."""
    ox, oy, oz = origin
    xs = ox + spacing * np.arange(width)
    zs = oz + spacing * np.arange(height)
    X, Z = np.meshgrid(xs, zs, indexing="xy")
    pos = np.stack([X, np.full_like(X, oy), Z], axis=-1).astype(np.float32)
    nrm = np.broadcast_to(np.asarray(normal, np.float32), pos.shape).copy()
    pr = np.full((height, width), prim, np.uint32)
    return GBuffer(pos, nrm, pr)


# --------------------------------------------------------------------------
# The named workloads
# --------------------------------------------------------------------------
AO_PLAIN_256 = dict(name="ao_256_boxes", mode="ao", width=256, height=256, radius=1.0, window_r=2,
                    scene_seed=1, sample_seed=1)
AO_1080P = dict(name="ao_1080p_terrain", mode="ao", width=1920, height=1080, radius=2.0, window_r=3,
                scene_seed=2, sample_seed=1)
SHADOW_1080P = dict(name="shadow_1080p_terrain", mode="shadow", width=1920, height=1080, radius=0.0,
                    window_r=3, scene_seed=2, sample_seed=1)


def boxes_camera(width: int = 256, height: int = 256) -> Camera:
    return pinhole((0.0, 12.0, -8.0), (0.0, 0.0, 0.0), width, height)


def terrain_camera(width: int = 1920, height: int = 1080) -> Camera:
    return pinhole((0.0, 45.0, -30.0), (0.0, 0.0, 12.0), width, height)


def terrain_light(hmax: float = 4.0) -> RectLight:
    """1 x 1 m rectangle 8 m above the highest terrain point, facing down."""
    return RectLight(np.array([0.0, hmax + 8.0, 12.0], np.float32), np.array([1.0, 0.0, 0.0], np.float32),
                     np.array([0.0, 0.0, 1.0], np.float32))


def two_lights(hmax: float = 4.0):
    """The terrain light and a second, 2 m x 1 m rectangle 10 m above the
    highest terrain point, rotated about the vertical and tilted (its edges
    are not axis-aligned), facing down: the shadows-of-several-lights input."""
    th = 0.5
    eu = np.array([np.cos(th), 0.1, np.sin(th)], np.float32) * np.float32(2.0)
    ev = np.cross(np.array([0.0, -1.0, 0.0]), eu.astype(np.float64))
    ev = (ev / np.linalg.norm(ev)).astype(np.float32)
    return [terrain_light(hmax), RectLight(np.array([25.0, hmax + 10.0, 30.0], np.float32), eu, ev)]


_CACHE: dict = {}


def workload(cfg: dict):
    """(scene, gbuffer, light_or_None) for one of the named workloads."""
    key = cfg["name"]
    if key in _CACHE:
        return _CACHE[key]
    if cfg["name"].startswith("ao_256"):
        scene = boxes_scene(cfg["scene_seed"])
        cam = boxes_camera(cfg["width"], cfg["height"])
    else:
        scene = terrain_scene(cfg["scene_seed"])
        cam = terrain_camera(cfg["width"], cfg["height"])
    gb = render_gbuffer(scene, cam)
    light = terrain_light() if cfg["mode"] == "shadow" else None
    _CACHE[key] = (scene, gb, light)
    return _CACHE[key]


# Batched workload: four terrain scenes and sixteen views of uneven size.
BATCH_SCENES = [dict(seed=10, cells=128, spheres=54), dict(seed=11, cells=256, spheres=375),
                dict(seed=2, cells=512, spheres=2000), dict(seed=13, cells=768, spheres=2560)]
BATCH_SIZES = [(640, 360), (2560, 1440), (960, 540), (1920, 1080), (1280, 720), (1600, 900), (640, 360),
               (2560, 1440), (1920, 1080), (960, 540), (1280, 720), (2560, 1440), (1600, 900), (640, 360),
               (1920, 1080), (1280, 720)]


def batch_scene(i: int) -> Scene:
    s = BATCH_SCENES[i]
    return terrain_scene(seed=s["seed"], cells=s["cells"], nspheres=s["spheres"])


def batch_views():
    """The sixteen views of the batched workload: view v shows scene v mod 4
    from orbit angle 2*pi*v/16 at BATCH_SIZES[v]; AO (R = 2 m) if v is even,
    else the 1 x 1 m shadow light.  Returns [(scene_index, camera, mode)]."""
    out = []
    for v, (W, H) in enumerate(BATCH_SIZES):
        out.append((v % 4, orbit_camera(v, 16, W, H), "ao" if v % 2 == 0 else "shadow"))
    return out
