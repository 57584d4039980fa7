"""Pins of the oracle's shadows under the solid-angle definition (App. on
that definition: Eq. reapp-shadow-definition-solid-angle, the estimator of
Eq. reapp-shadow-solid-angle-estimator with the factor C_Omega of Eq.
reapp-shadow-solid-angle-mis-factor).

The emitter's solid angle is pinned to the closed form for a rectangle seen
on its axis and to a cell quadrature of cos / r^2 dA off axis; the factor
C_Omega to the identity C_Omega p_Sh = J_{Omega->S} / Omega_A of Eq.
reapp-shadow-solid-angle-mis-numerator and to its mean over the light; the
estimators to FP64 quadrature of the definition (unbiased and no-reuse
converge, biased does not where first-hit consistency fails)."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w


def _light(Hl=2.0, Lu=1.0, Lv=1.0, cx=0.0, cz=0.0):
    return w.RectLight(np.array([cx, Hl, cz], np.float32), np.array([Lu, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, Lv], np.float32))


def _cells(light, n):
    """Cell centres of an n x n midpoint grid over the light and the cell area."""
    la = light.as_array().astype(np.float64)
    c, eu, ev = la[0:3], la[3:6], la[6:9]
    u = (np.arange(n) + 0.5) / n - 0.5
    U, V = np.meshgrid(u, u, indexing="ij")
    Y = c + U[..., None] * eu + V[..., None] * ev
    area = np.linalg.norm(np.cross(eu, ev))
    return Y.reshape(-1, 3), area / (n * n)


def _quad_solid_angle(o, n, light, ncell=1500, front_only=False):
    Y, dA = _cells(light, ncell)
    d = Y - np.asarray(o, np.float64)
    r2 = (d * d).sum(1)
    nl = np.array([0.0, -1.0, 0.0])
    wgt = -(d @ nl) / np.sqrt(r2) / r2 * dA
    if front_only:
        wgt = wgt * ((d @ np.asarray(n, np.float64)) > 0.0)
    return wgt.sum()


@pytest.mark.parametrize("a,b,d", [(1.0, 1.0, 2.0), (2.0, 0.5, 0.7), (0.2, 0.3, 10.0)])
def test_rectangle_on_axis_closed_form(a, b, d):
    light = _light(Hl=d, Lu=a, Lv=b)
    all_, front = oracle.solid_angles([0.0, 0.0, 0.0], [0.0, 1.0, 0.0], light)
    a, b, d = (float(np.float32(v)) for v in (a, b, d))  # the light is given in FP32
    ref = 4.0 * np.arcsin(a * b / np.sqrt((a * a + 4 * d * d) * (b * b + 4 * d * d)))
    assert all_ == pytest.approx(ref, rel=1e-12)
    assert front == pytest.approx(ref, rel=1e-12)  # the whole light is in front


@pytest.mark.parametrize("o,n", [([0.7, 0.0, -0.4], [0.0, 1.0, 0.0]),
                                 ([0.3, 0.5, 0.2], [0.6, 0.8, 0.0]),
                                 ([-0.2, 1.2, 0.1], [0.0, 0.6, -0.8])])
def test_solid_angle_matches_cell_quadrature(o, n):
    light = _light()
    all_, front = oracle.solid_angles(o, n, light)
    assert all_ == pytest.approx(_quad_solid_angle(o, n, light), rel=2e-6)
    # the clipped part converges at first order in the cell size along the cut
    assert front == pytest.approx(_quad_solid_angle(o, n, light, front_only=True), rel=3e-3)
    assert 0.0 < front <= all_


def test_tangent_plane_halves_partition_the_emitter():
    light = _light()
    o = np.array([0.1, 0.9, -0.2])
    for th in np.linspace(0.2, 2.9, 7):
        n = np.array([np.cos(th), np.sin(th) * 0.6, np.sin(th) * 0.8])
        a1, f1 = oracle.solid_angles(o, n, light)
        a2, f2 = oracle.solid_angles(o, -n, light)
        assert a1 == a2
        assert f1 + f2 == pytest.approx(a1, rel=1e-12)


def test_receiver_behind_or_in_the_light_plane_sees_nothing():
    light = _light()
    assert oracle.solid_angles([0.0, 3.0, 0.0], [0.0, -1.0, 0.0], light) == (0.0, 0.0)
    assert oracle.solid_angles([0.3, 2.0, 0.0], [0.0, 1.0, 0.0], light) == (0.0, 0.0)


@pytest.mark.parametrize("tilt", [0.0, 0.5])
def test_factor_times_density_is_the_solid_angle_integrand(tilt):
    # C_Omega p_Sh = F_Sh,Omega = J_{Omega->S}(x, z) / Omega_A(x) for a pair
    # inside the support (Eqs. reapp-shadow-solid-angle-integrand and
    # reapp-shadow-solid-angle-mis-numerator), with J_{Omega->S} = <n_z,
    # w_{z->x}> / |x - z|^2 and p_Sh carrying its 1/Area.
    light = _light()
    rng = np.random.default_rng(3)
    o = np.array([0.05, 0.0, -0.1])
    n = np.array([np.sin(tilt), np.cos(tilt), 0.0])
    all_, _ = oracle.solid_angles(o, n, light)
    checked = 0
    for _ in range(200):
        y = np.array([rng.uniform(-0.5, 0.5), 2.0, rng.uniform(-0.5, 0.5)])
        t = rng.uniform(0.1, 0.9)
        z = o + t * (y - o)
        nz = rng.normal(size=3)
        nz /= np.linalg.norm(nz)
        if nz @ (o - z) < 0:
            nz = -nz
        p = oracle.density_shadow(o, n, z, nz, light)
        if p == 0.0:
            continue
        wzx = (o - z) / np.linalg.norm(o - z)
        ref = (nz @ wzx) / ((o - z) @ (o - z)) / all_
        assert oracle.sa_factor(o, n, z, light) * p == pytest.approx(ref, rel=1e-12)
        checked += 1
    assert checked > 100


def test_factor_averages_to_the_front_fraction():
    # (1/Area) \int_{front} C_Omega(x, y) dA(y) = Omega_front / Omega_A: the
    # no-reuse estimator F_Omega - C_Omega [blocked] is unbiased.
    light = _light()
    o = np.array([0.2, 0.4, 0.1])
    n = np.array([0.5, 0.7, 0.5])
    n /= np.linalg.norm(n)
    all_, front = oracle.solid_angles(o, n, light)
    Y, dA = _cells(light, 300)
    acc = 0.0
    for y in Y:
        if (y - o) @ n > 0.0:
            acc += oracle.sa_factor(o, n, o + 0.5 * (y - o), light)
    area = 1.0
    assert acc * dA / area == pytest.approx(front / all_, rel=2e-3)


# --------------------------------------------------------------------------
# Estimators against quadrature of the definition
# --------------------------------------------------------------------------
M = 4096
TARGETS = [(x, y) for y in (3, 4) for x in (4, 5, 6, 7)]
CONFIGS = [("window", 1), ("window", 3), ("group", 2), ("group", 8)]
SIGMA_REF = 1e-3
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
        zs.append((m - refs[(x, y)]) / np.sqrt(var / M + SIGMA_REF ** 2))
    return np.array(zs)


@pytest.fixture(scope="module", params=["flat", "tilted"])
def sa_inconsistent(request):
    # the shadow fixture of the area-definition tests: a high plate whose
    # occluders are hidden from inner receivers by a low strip
    light = _light()
    sc = _oscene([scenes.plate_y(1.0, -0.5, 0.02, -3, 3), scenes.plate_y(0.1, -0.12, -0.06, -3, 3)])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    if request.param == "tilted":
        th = np.arctan2(1.0, -0.1)
        gb.nrm[:] = np.array([np.sin(th), np.cos(th), 0.0], np.float32)
    o, _, _ = oracle.samples(gb, oracle.params("shadow_sa", "none", light=light))
    refs = {(x, y): sc.shadow_sa_quadrature(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), light,
                                            ign=0, ngrid=1024) for (x, y) in TARGETS}
    return sc, gb, refs, light, request.param


def test_open_plane_is_the_front_fraction():
    sc = _oscene([])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    light = _light()
    for est in ("none", "biased", "unbiased"):
        _, r = oracle.frame(sc, gb, oracle.params("shadow_sa", est, "window", radius=2, light=light, seed=5))
        assert np.allclose(r.value, 1.0)  # every receiver faces the whole light; nothing blocks


def test_quadrature_differs_from_the_area_definition(sa_inconsistent):
    # the two definitions weight the light differently (cos/r^2 vs area)
    sc, gb, refs, light, kind = sa_inconsistent
    o, _, _ = oracle.samples(gb, oracle.params("shadow_sa", "none", light=light))
    diffs = [abs(refs[(x, y)] - sc.shadow_quadrature(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64),
                                                       light, ign=0, ngrid=1024)) for (x, y) in TARGETS]
    assert max(diffs) > 5e-3


def test_sa_no_reuse_converges(sa_inconsistent):
    sc, gb, refs, light, kind = sa_inconsistent
    z = _z_scores(sc, gb, oracle.params("shadow_sa", "none", light=light, seed=7), refs)
    assert np.abs(z).max() < Z_MAX, z


@pytest.mark.parametrize("pattern,size", CONFIGS)
def test_sa_unbiased_converges(sa_inconsistent, pattern, size):
    sc, gb, refs, light, kind = sa_inconsistent
    pu = oracle.params("shadow_sa", "unbiased", pattern, radius=size, group_n=size, light=light, seed=7)
    zu = _z_scores(sc, gb, pu, refs)
    assert np.abs(zu).max() < Z_MAX, zu
    if kind == "flat":
        pb = oracle.params("shadow_sa", "biased", pattern, radius=size, group_n=size, light=light, seed=7,
                           dark_guard=False)
        zb = _z_scores(sc, gb, pb, refs)
        assert np.abs(zb).max() > 6.0, zb
