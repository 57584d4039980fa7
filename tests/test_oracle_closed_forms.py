"""Closed-form pins of the oracle: quadrature references of AO (Sec. 3.2
Eq. ao-hemisphere) and normalised shadow (Sec. 3.3 Eq. shadow-area) against
textbook geometry, the induced densities (Eqs. ao-pdf, shadow-pdf with the
Jacobians of Eqs. ao-jacobian, shadow-jacobian) integrated over occluder
planes, and the front fraction F_i against hand-computed clips."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w

O = np.array([0.0, 0.0, 0.0])
UP = np.array([0.0, 1.0, 0.0])


def _scene(parts):
    s = scenes.build([scenes.FLOOR] + parts)
    return oracle.Scene(s.V, s.F, grid=True)


def test_open_plane_ao_and_shadow_are_one():
    sc = _scene([])
    assert sc.ao_quadrature(O, UP, 1.0, ign=0, nstrata=128) == 1.0
    light = w.terrain_light()
    assert sc.shadow_quadrature(O, UP, light, ign=0, ngrid=64) == 1.0


@pytest.mark.parametrize("d", [1e-3, 0.3, 0.7])
def test_wall_circular_segment(d):
    # Wall X = d beside an up-facing receiver: directions with Malley disc
    # coordinate alpha >= d/R reach it within R, a circular segment of the disc.
    R = 1.0
    sc = _scene([scenes.wall_x(d)])
    a = d / R
    closed = 1.0 - (np.arccos(a) - a * np.sqrt(1 - a * a)) / np.pi
    q = sc.ao_quadrature(O, UP, R, ign=0, nstrata=1024)
    assert abs(q - closed) < 2e-3, (q, closed)


def test_foot_of_infinite_wall_is_one_half():
    sc = _scene([scenes.wall_x(1e-6, y1=1e4, z0=-1e4, z1=1e4)])
    q = sc.ao_quadrature(O, UP, 1e3, ign=0, nstrata=1024)
    assert abs(q - 0.5) < 2e-3
    # the occlusion convention (1 - AO) gives the same value
    assert abs((1 - q) - 0.5) < 2e-3


@pytest.mark.parametrize("h", [0.25, 0.6, 0.9])
def test_ceiling(h):
    # A ceiling at height h <= R is reached within R iff cos(theta) >= h/R,
    # which cosine sampling does with probability 1 - (h/R)^2.
    R = 1.0
    sc = _scene([scenes.plate_y(h, -50, 50, -50, 50)])
    q = sc.ao_quadrature(O, UP, R, ign=0, nstrata=1024)
    assert abs(q - (h / R) ** 2) < 2e-3


def test_lambert_disc_limit():
    # Lambert's polygon formula for a fine regular polygon tends to the
    # coaxial disc's form factor rho^2 / (h^2 + rho^2).
    h, rho = 0.7, 0.5
    ang = np.linspace(0, 2 * np.pi, 2049)[:-1]
    verts = [(rho * np.cos(t), h, rho * np.sin(t)) for t in ang]
    ff = scenes.lambert_polygon_ff(O, UP, verts)
    assert abs(ff - rho ** 2 / (h ** 2 + rho ** 2)) < 1e-5


@pytest.mark.parametrize("n_sides", [4, 7, 64])
def test_polygon_occluder_lambert(n_sides):
    h, rho = 0.6, 0.45
    ang = np.linspace(0, 2 * np.pi, n_sides + 1)[:-1] + 0.3
    verts = [(rho * np.cos(t) + 0.1, h, rho * np.sin(t)) for t in ang]
    V, F = scenes.polygon_fan((0.1, h, 0.0), verts)
    sc = _scene([(V, F)])
    q = sc.ao_quadrature(O, UP, 10.0, ign=0, nstrata=1024)
    ff = scenes.lambert_polygon_ff(O, UP, verts)
    assert abs((1 - q) - ff) < 2e-3, (1 - q, ff)


def _light(Hl, L, cx=0.0, cz=0.0):
    return w.RectLight(np.array([cx, Hl, cz], np.float32), np.array([L, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, L], np.float32))


@pytest.mark.parametrize("s_occ", [0.1, 0.25, 0.6])
def test_parallel_square_occluder_shadow(s_occ):
    # Centred square of side s at height h under a parallel square light of
    # side L at height H: its shadow covers a centred square of side s H / h
    # of the light, so Shadow = 1 - min(1, s H / (h L))^2.
    h, Hl, L = 1.0, 3.0, 1.0
    sc = _scene([scenes.plate_y(h, -s_occ / 2, s_occ / 2, -s_occ / 2, s_occ / 2)])
    q = sc.shadow_quadrature(O, UP, _light(Hl, L), ign=0, ngrid=512)
    closed = 1 - min(1.0, s_occ * Hl / (h * L)) ** 2
    assert abs(q - closed) < 4e-3, (q, closed)


def test_off_centre_rectangle_occluder_shadow():
    h, Hl, L = 1.0, 4.0, 1.0
    x0, x1, z0, z1 = 0.02, 0.3, -0.05, 0.08
    sc = _scene([scenes.plate_y(h, x0, x1, z0, z1)])
    q = sc.shadow_quadrature(O, UP, _light(Hl, L), ign=0, ngrid=512)
    k = Hl / h
    ox = max(0.0, min(x1 * k, 0.5) - max(x0 * k, -0.5))
    oz = max(0.0, min(z1 * k, 0.5) - max(z0 * k, -0.5))
    assert abs(q - (1 - ox * oz / L ** 2)) < 4e-3


def test_receiver_facing_away_is_dark():
    sc = _scene([])
    assert sc.shadow_quadrature(O, -UP, _light(3.0, 1.0), ign=0, ngrid=64) == 0.0


def test_front_fraction_clips():
    light = _light(2.0, 1.0)
    assert oracle.front_fraction(O, UP, light) == pytest.approx(1.0, abs=1e-12)
    assert oracle.front_fraction(O, -UP, light) == 0.0
    # tangent plane through the light's centre line: half
    assert oracle.front_fraction(O, [1.0, 0.0, 0.0], light) == pytest.approx(0.5, abs=1e-12)
    # tilted about z: front part x > -H cot(theta) -> 0.5 + H cot(theta)
    th = np.arctan(10.0)
    n = np.array([np.sin(th), np.cos(th), 0.0])
    assert oracle.front_fraction(O, n, light) == pytest.approx(0.5 + 2.0 / 10.0, abs=1e-12)
    # tilted about the diagonal: front part x + z > k cuts a corner triangle
    k = 0.6
    cot = k / (np.sqrt(2) * 2.0)
    th = np.arctan(1 / cot)
    n = np.array([-np.sin(th) / np.sqrt(2), np.cos(th), -np.sin(th) / np.sqrt(2)])
    # front: -(x+z) sin/sqrt2 + H cos > 0 -> x + z < k  => area 1 - (1-k)^2/2
    assert oracle.front_fraction(O, n, light) == pytest.approx(1 - (1 - k) ** 2 / 2, abs=1e-12)
    # receiver behind the light's emitting face
    assert oracle.front_fraction([0.0, 3.0, 0.0], UP, light) == 0.0


@pytest.mark.parametrize("h,R", [(0.3, 1.0), (0.8, 1.0), (0.5, 2.0)])
def test_ao_density_integrates_over_ceiling(h, R):
    # \int p_AO dmu over a ceiling at height h (normal facing the receiver)
    # is the probability that a cosine ray reaches it within R: 1 - (h/R)^2.
    nz = np.array([0.0, -1.0, 0.0])
    rmax = np.sqrt(R * R - h * h)
    n = 401
    xs = (np.arange(n) + 0.5) / n * 2 * rmax - rmax
    cell = (2 * rmax / n) ** 2
    acc = 0.0
    for x in xs:
        for z in xs:
            if x * x + z * z <= rmax * rmax * 1.02:
                acc += oracle.density_ao(O, UP, [x, h, z], nz, R)
    assert abs(acc * cell - (1 - (h / R) ** 2)) < 5e-3


@pytest.mark.parametrize("tilt", [0.0, 0.2])
def test_shadow_density_integrates_to_front_fraction(tilt):
    # \int p_Sh dmu over an occluder plane covering the light's projection is
    # the probability that a light sample is in front of the receiver and
    # blocked by the plane: F_i.
    Hl, L, h = 2.0, 1.0, 0.8
    light = _light(Hl, L)
    th = np.arctan(1 / tilt) if tilt > 0 else 0.0
    n = np.array([np.sin(th), np.cos(th), 0.0]) if tilt > 0 else UP
    F = oracle.front_fraction(O, n, light)
    nz = np.array([0.0, -1.0, 0.0])
    half = L * h / Hl / 2
    m = 300
    xs = (np.arange(m) + 0.5) / m * 2.4 * half - 1.2 * half
    cell = (2.4 * half / m) ** 2
    acc = 0.0
    for x in xs:
        for z in xs:
            acc += oracle.density_shadow(O, n, [x, h, z], nz, light)
    assert abs(acc * cell - F) < 1e-2, (acc * cell, F)
    if tilt > 0:
        assert F == pytest.approx(0.5 + Hl * tilt, abs=1e-12)
