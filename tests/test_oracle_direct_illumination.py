"""Pins of the oracle's occluder-domain direct illumination (the appendix
deriving Eq. reapp-di-occluder-domain-compact, with the MIS estimator of Eq.
reapp-di-general-mis-estimator and factor of Eq.
reapp-di-general-mis-factor), for a Lambertian receiver under a uniform
one-sided emitter, in units of rho L_e / pi (the visible irradiance of a
unit-radiance light).

The unshadowed term U (Lambert's polygon formula over the light clipped by
the tangent plane) is pinned to the textbook form factor from a point to a
parallel rectangle and to a cell quadrature for tilted receivers; the factor
C_DI to the identity C_DI p_Sh = cos+_x <n_z, w_{z->x}> / |x - z|^2 (the
surface-domain integrand of Eq. reapp-di-blocked-occ) and to its mean over
the light; the estimators to an FP64 quadrature of Eq. reapp-di-area-compact
(no reuse and unbiased converge, biased does not)."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w


def _light(Hl=2.0, Lu=1.0, Lv=1.0, cx=0.0, cz=0.0):
    return w.RectLight(np.array([cx, Hl, cz], np.float32), np.array([Lu, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, Lv], np.float32))


def _corner_ff(a, b, d):
    """Form factor from a differential area to a parallel a x b rectangle with
    one corner above it at height d (the textbook closed form)."""
    X, Y = a / d, b / d
    return (X / np.sqrt(1 + X * X) * np.arctan(Y / np.sqrt(1 + X * X))
            + Y / np.sqrt(1 + Y * Y) * np.arctan(X / np.sqrt(1 + Y * Y))) / (2 * np.pi)


@pytest.mark.parametrize("px,pz,d,Lu,Lv", [(0.0, 0.0, 2.0, 1.0, 1.0), (0.2, -0.1, 1.5, 1.0, 1.0),
                                           (0.05, 0.3, 0.8, 2.0, 1.0)])
def test_unshadowed_term_is_the_rectangle_form_factor(px, pz, d, Lu, Lv):
    light = _light(Hl=d, Lu=Lu, Lv=Lv)
    Lu, Lv, d = (float(np.float32(v)) for v in (Lu, Lv, d))
    E = oracle.emitter_irradiance([px, 0.0, pz], [0.0, 1.0, 0.0], light)
    # the foot point splits the light into four rectangles with a corner above it
    xs = (Lu / 2 - px, Lu / 2 + px)
    zs = (Lv / 2 - pz, Lv / 2 + pz)
    ref = np.pi * sum(_corner_ff(a, b, d) for a in xs for b in zs)
    assert E == pytest.approx(ref, rel=1e-12)


def _cells(light, n):
    la = light.as_array().astype(np.float64)
    c, eu, ev = la[0:3], la[3:6], la[6:9]
    u = (np.arange(n) + 0.5) / n - 0.5
    U, V = np.meshgrid(u, u, indexing="ij")
    Y = c + U[..., None] * eu + V[..., None] * ev
    return Y.reshape(-1, 3), np.linalg.norm(np.cross(eu, ev)) / (n * n)


@pytest.mark.parametrize("o,n", [([0.3, 0.5, 0.2], [0.6, 0.8, 0.0]), ([-0.2, 1.2, 0.1], [0.0, 0.6, -0.8]),
                                 ([0.1, 0.9, -0.2], [0.95, 0.1, 0.3])])
def test_unshadowed_term_matches_cell_quadrature(o, n):
    light = _light()
    n = np.asarray(n, np.float64) / np.linalg.norm(n)
    Y, dA = _cells(light, 1500)
    d = Y - np.asarray(o, np.float64)
    r2 = (d * d).sum(1)
    cx = np.maximum(d @ n, 0.0) / np.sqrt(r2)
    cy = d[:, 1] / np.sqrt(r2)  # the light faces -y
    ref = (cx * cy / r2).sum() * dA
    assert oracle.emitter_irradiance(o, n, light) == pytest.approx(ref, rel=2e-4)


def test_factor_times_density_is_the_surface_integrand():
    light = _light()
    rng = np.random.default_rng(5)
    o = np.array([0.05, 0.0, -0.1])
    n = np.array([0.3, 0.95, 0.0])
    n /= np.linalg.norm(n)
    checked = 0
    for _ in range(200):
        y = np.array([rng.uniform(-0.5, 0.5), 2.0, rng.uniform(-0.5, 0.5)])
        z = o + rng.uniform(0.1, 0.9) * (y - o)
        nz = rng.normal(size=3)
        nz /= np.linalg.norm(nz)
        if nz @ (o - z) < 0:
            nz = -nz
        p = oracle.density_shadow(o, n, z, nz, light)
        if p == 0.0:
            continue
        wxz = (z - o) / np.linalg.norm(z - o)
        ref = max(n @ wxz, 0.0) * (nz @ -wxz) / ((z - o) @ (z - o))
        assert oracle.di_factor(o, n, z, light) * p == pytest.approx(ref, rel=1e-12)
        checked += 1
    assert checked > 100


def test_factor_averages_to_the_unshadowed_term():
    light = _light()
    o = np.array([0.2, 0.4, 0.1])
    n = np.array([0.5, 0.7, 0.5])
    n /= np.linalg.norm(n)
    Y, dA = _cells(light, 300)
    acc = 0.0
    for y in Y:
        if (y - o) @ n > 0.0:
            acc += oracle.di_factor(o, n, o + 0.5 * (y - o), light)
    assert acc * dA == pytest.approx(oracle.emitter_irradiance(o, n, light), rel=2e-3)


M = 4096
TARGETS = [(x, y) for y in (3, 4) for x in (4, 5, 6, 7)]
Z_MAX = 4.0


def _oscene(parts):
    s = scenes.build([scenes.FLOOR] + parts)
    return oracle.Scene(s.V, s.F, grid=True)


def _z_scores(sc, gb, p, refs):
    s, s2 = oracle.render(sc, gb, p, M, region=(4, 3, 8, 5))
    zs = []
    for (x, y) in TARGETS:
        m = s[y, x] / M
        var = max(s2[y, x] / M - m * m, 0.0)
        zs.append((m - refs[(x, y)]) / np.sqrt(var / M + (1e-3 * refs[(x, y)] + 1e-6) ** 2))
    return np.array(zs)


@pytest.fixture(scope="module", params=["flat", "tilted"])
def di_inconsistent(request):
    light = _light()
    sc = _oscene([scenes.plate_y(1.0, -0.5, 0.02, -3, 3), scenes.plate_y(0.1, -0.12, -0.06, -3, 3)])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    if request.param == "tilted":
        th = np.arctan2(1.0, -0.1)
        gb.nrm[:] = np.array([np.sin(th), np.cos(th), 0.0], np.float32)
    o, _, _ = oracle.samples(gb, oracle.params("di", "none", light=light))
    refs = {(x, y): sc.di_quadrature(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), light, ign=0,
                                     ngrid=1024) for (x, y) in TARGETS}
    return sc, gb, refs, light, request.param


def test_open_plane_is_the_unshadowed_term():
    sc = _oscene([])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    light = _light()
    o, _, _ = oracle.samples(gb, oracle.params("di", "none", light=light))
    for est in ("none", "biased", "unbiased"):
        _, r = oracle.frame(sc, gb, oracle.params("di", est, "window", radius=2, light=light, seed=5))
        for (x, y) in TARGETS:
            U = oracle.emitter_irradiance(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), light)
            assert r.value[y, x] == pytest.approx(U, rel=1e-12)


def test_di_no_reuse_converges(di_inconsistent):
    sc, gb, refs, light, kind = di_inconsistent
    z = _z_scores(sc, gb, oracle.params("di", "none", light=light, seed=7), refs)
    assert np.abs(z).max() < Z_MAX, z


@pytest.mark.parametrize("pattern,size", [("window", 1), ("window", 3), ("group", 2), ("group", 8)])
def test_di_unbiased_converges(di_inconsistent, pattern, size):
    sc, gb, refs, light, kind = di_inconsistent
    zu = _z_scores(sc, gb, oracle.params("di", "unbiased", pattern, radius=size, group_n=size, light=light, seed=7),
                   refs)
    assert np.abs(zu).max() < Z_MAX, zu
    if kind == "flat":
        pb = oracle.params("di", "biased", pattern, radius=size, group_n=size, light=light, seed=7, dark_guard=False)
        zb = _z_scores(sc, gb, pb, refs)
        assert np.abs(zb).max() > 6.0, zb
