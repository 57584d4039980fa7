"""Pins of the oracle's shadows and direct illumination sampled from a general
emitter-area density p_A(y' | x) (App., general area-domain sampling density:
the induced density p_A(y' | x) J chi_A Occ and the estimator factors divided
by Area p_A).  The density built is the receiver-dependent bilinear one: the
corner weights 1 / |o - y_k|^3, the shape of the solid-angle density
cos(theta_y) / |o - y|^2, interpolated bilinearly over the rectangle.

The density is pinned to the solid-angle shape at the corners (computed here
from the geometry), to bilinearity and to unit mass; the FP32 sampler to the
density by a chi-square test of its histogram; the one-sample weight to
1 / (Area p_A) at the sample's own point; N = 1 reuse to no reuse; the
consistent scene to biased == unbiased; and the no-reuse and unbiased
estimators of all three quantities to FP64 quadrature of their definitions,
which do not depend on the sampling density."""
import numpy as np
import pytest
from scipy import stats

import oracle
import scenes
import workloads as w


def _light(Hl=0.6, L=1.0, cx=0.0, cz=0.0, pdf=1):
    # facing down: e_u x e_v = x cross z = -y
    return w.RectLight(np.array([cx, Hl, cz], np.float32), np.array([L, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, L], np.float32), pdf)


def _tilted_light():
    # rotated in its plane and tilted, so that a, b and the corner order matter
    c = np.array([0.3, 1.2, -0.2])
    eu = np.array([0.9, 0.15, 0.4])
    t = np.array([-0.4, 0.1, 0.9])
    ev = t - eu * (t @ eu) / (eu @ eu)
    ev = ev / np.linalg.norm(ev) * 0.7
    if np.cross(eu, ev)[1] > 0:
        ev = -ev
    return w.RectLight(c.astype(np.float32), eu.astype(np.float32), ev.astype(np.float32), 1)


def _frame(light):
    la = light.as_array().astype(np.float64)
    return la[0:3], la[3:6], la[6:9]


CORNERS = [(-0.5, -0.5), (0.5, -0.5), (-0.5, 0.5), (0.5, 0.5)]


@pytest.mark.parametrize("light,o", [(_light(), np.array([0.45, 0.0, 0.3])),
                                     (_light(), np.array([-0.2, 0.3, 0.05])),
                                     (_tilted_light(), np.array([0.1, 0.0, 0.2])),
                                     (_tilted_light(), np.array([1.0, -0.5, -0.6]))])
def test_density_has_the_solid_angle_shape_at_the_corners(light, o):
    c, eu, ev = _frame(light)
    nl = np.cross(eu, ev)
    nl /= np.linalg.norm(nl)
    q = np.array([oracle.light_q(o, light, a, b) for (a, b) in CORNERS])
    sa = []
    for (a, b) in CORNERS:
        y = c + a * eu + b * ev
        d = np.linalg.norm(o - y)
        sa.append(abs(nl @ (o - y)) / d / d ** 2)  # cos(theta_y) / |o - y|^2
    sa = np.array(sa)
    np.testing.assert_allclose(q / q[0], sa / sa[0], rtol=1e-12)
    assert q.max() / q.min() > 1.2  # not the uniform density
    # bilinear: the centre and the edge midpoints are the means of the corners
    assert oracle.light_q(o, light, 0.0, 0.0) == pytest.approx(q.mean(), rel=1e-13)
    assert oracle.light_q(o, light, 0.0, -0.5) == pytest.approx((q[0] + q[1]) / 2, rel=1e-13)
    assert oracle.light_q(o, light, 0.5, 0.0) == pytest.approx((q[1] + q[3]) / 2, rel=1e-13)
    # unit mass (the midpoint rule is exact for a bilinear function)
    g = (np.arange(16) + 0.5) / 16 - 0.5
    assert np.mean([[oracle.light_q(o, light, a, b) for a in g] for b in g]) == pytest.approx(1.0, rel=1e-12)


def test_receiver_on_the_axis_sees_the_uniform_density():
    light = _tilted_light()
    c, eu, ev = _frame(light)
    nl = np.cross(eu, ev)
    o = c + 0.8 * nl / np.linalg.norm(nl)
    rng = np.random.default_rng(3)
    for a, b in rng.uniform(-0.5, 0.5, (10, 2)):
        assert oracle.light_q(o, light, a, b) == pytest.approx(1.0, rel=1e-6)


def _sample_uv(light, o_pt, n=64, spp=8):
    """(u, v) in [0, 1]^2 of the FP32 samples of n x n pixels that all sit at o_pt."""
    gb = scenes.floor_grid(n, n, 0.0, x0=float(o_pt[0]), z0=float(o_pt[2]))
    gb.pos[..., 1] = np.float32(o_pt[1])
    c, eu, ev = _frame(light)
    uv = []
    for s in range(spp):
        o, d, kind = oracle.samples(gb, oracle.params("shadow", "none", light=light, seed=11, sample=s))
        y = (o.astype(np.float64) + d.astype(np.float64)).reshape(-1, 3)
        assert (kind == 0).all()
        uv.append(np.stack([(y - c) @ eu / (eu @ eu) + 0.5, (y - c) @ ev / (ev @ ev) + 0.5], 1))
    o0 = o[0, 0].astype(np.float64)
    return np.concatenate(uv), o0


@pytest.mark.parametrize("light,o_pt", [(_light(Hl=0.5), (0.45, 0.0, 0.3)), (_light(Hl=0.5), (0.0, 0.0, 0.0)),
                                        (_tilted_light(), (0.1, 0.0, 0.2))])
def test_sampler_draws_from_the_density(light, o_pt):
    uv, o = _sample_uv(light, o_pt)
    assert (uv >= -1e-6).all() and (uv <= 1 + 1e-6).all()
    K = 8
    cnt, _, _ = np.histogram2d(uv[:, 0], uv[:, 1], bins=K, range=[[0, 1], [0, 1]])
    mid = (np.arange(K) + 0.5) / K - 0.5
    # cell probability = q at the cell centre / K^2 (exact for a bilinear q)
    prob = np.array([[oracle.light_q(o, light, a, b) for b in mid] for a in mid]) / K ** 2
    assert prob.sum() == pytest.approx(1.0, rel=1e-9)
    exp = prob * len(uv)
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, K * K - 1) > 1e-4, chi2
    # and a uniform histogram is rejected where the density is not uniform
    if prob.max() / prob.min() > 2:
        chi2u = ((cnt - len(uv) / K ** 2) ** 2 / (len(uv) / K ** 2)).sum()
        assert stats.chi2.sf(chi2u, K * K - 1) < 1e-12


def test_one_sample_weight_is_the_inverse_density():
    # a plate over the whole floor blocks every sample: no reuse gives
    # F - 1 / (Area p_A(y | x)) at the sample's own light point (F = 1 below)
    light = _light(Hl=0.5)
    sc = oracle.Scene(*_parts([scenes.plate_y(0.25, -3, 3, -3, 3)]), grid=True)
    gb = scenes.floor_grid(10, 8, 0.07, x0=-0.3, z0=-0.25)
    p = oracle.params("shadow", "none", light=light, seed=5)
    rec, res = oracle.frame(sc, gb, p)
    assert (rec.hit != oracle.MISS).all()
    o, d, _ = oracle.samples(gb, p)
    c, eu, ev = _frame(light)
    y = o.astype(np.float64) + d.astype(np.float64)
    for iy in range(gb.height):
        for ix in range(gb.width):
            a = (y[iy, ix] - c) @ eu / (eu @ eu)
            b = (y[iy, ix] - c) @ ev / (ev @ ev)
            q = oracle.light_q(o[iy, ix].astype(np.float64), light, a, b)
            assert res.value[iy, ix] == pytest.approx(1.0 - 1.0 / q, rel=1e-5, abs=1e-6)
    assert res.value.min() < -0.2 and res.value.max() > 0.2  # far from F - 1 = 0


def _parts(parts):
    s = scenes.build([scenes.FLOOR] + parts)
    return s.V, s.F


@pytest.mark.parametrize("mode", ["shadow", "shadow_sa", "di"])
def test_single_pixel_sets_are_no_reuse(mode):
    light = _light(cx=0.1, cz=0.05)
    sc = oracle.Scene(*_parts([scenes.plate_y(0.3, -0.5, 0.05, -3, 3), scenes.plate_y(0.08, -0.12, -0.06, -3, 3)]),
                      grid=True)
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    rec, r0 = oracle.frame(sc, gb, oracle.params(mode, "none", light=light, seed=3))
    assert (rec.hit != oracle.MISS).any() and (rec.hit == oracle.MISS).any()
    for est in ("biased", "unbiased"):
        r1 = oracle.reuse(sc, gb, oracle.params(mode, est, "window", radius=0, light=light, seed=3,
                                                dark_guard=False), rec)
        assert np.array_equal(r1.value, r0.value), est


@pytest.mark.parametrize("mode", ["shadow", "shadow_sa", "di"])
def test_consistent_scene_biased_equals_unbiased(mode):
    light = _light(cx=0.1)
    sc = oracle.Scene(*_parts([scenes.plate_y(0.3, -0.2, 0.15, -3, 3)]), grid=True)
    gb = scenes.floor_grid(16, 12, 0.04, x0=-0.3, z0=-0.2)
    for pattern, size in [("window", 3), ("group", 8)]:
        pb = oracle.params(mode, "biased", pattern, radius=size, group_n=size, light=light, seed=9, dark_guard=False)
        pu = oracle.params(mode, "unbiased", pattern, radius=size, group_n=size, light=light, seed=9)
        rec, rb = oracle.frame(sc, gb, pb)
        ru = oracle.reuse(sc, gb, pu, rec)
        assert np.array_equal(rb.value, ru.value)
        assert (rec.hit != oracle.MISS).mean() > 0.2


def test_parameter_checks():
    with pytest.raises(ValueError):
        oracle.params("shadow", "biased", light=[_light(), _light(cx=1.0)])
    with pytest.raises(ValueError):
        oracle.params("shadow", "filter", light=_light())
    assert oracle.params("shadow", "biased", light=_light()).light_pdf == 1
    assert oracle.params("shadow", "biased", light=_light(pdf=0)).light_pdf == 0


# --------------------------------------------------------------------------
# Unbiasedness under the bilinear density: the targets are the definitions'
# FP64 quadratures (independent of how the light is sampled).
# --------------------------------------------------------------------------
M = 4096
TARGETS = [(x, y) for y in (3, 4) for x in (4, 5, 6, 7)]
SIGMA_REF = 1e-3
Z_MAX = 4.0


def _z_scores(sc, gb, p, refs):
    s, s2 = oracle.render(sc, gb, p, M, region=(4, 3, 8, 5))
    zs = []
    for (x, y) in TARGETS:
        m = s[y, x] / M
        var = max(s2[y, x] / M - m * m, 0.0)
        zs.append((m - refs[(x, y)]) / np.sqrt(var / M + SIGMA_REF ** 2))
    return np.array(zs)


@pytest.fixture(scope="module", params=["shadow", "shadow_sa", "di"])
def low_light(request):
    # a low light off the receivers' centre (the density varies by ~2.5x over
    # it), a plate that half covers it and a low strip that hides part of
    # the plate from some receivers (first-hit consistency fails)
    mode = request.param
    light = _light(Hl=0.6, cx=0.15, cz=0.1)
    sc = oracle.Scene(*_parts([scenes.plate_y(0.3, -0.5, 0.1, -3, 3), scenes.plate_y(0.08, -0.12, -0.06, -3, 3)]),
                      grid=True)
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    o, _, _ = oracle.samples(gb, oracle.params(mode, "none", light=light))
    quad = {"shadow": sc.shadow_quadrature, "shadow_sa": sc.shadow_sa_quadrature, "di": sc.di_quadrature}[mode]
    refs = {(x, y): quad(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), light, ign=0, ngrid=1024)
            for (x, y) in TARGETS}
    qs = [oracle.light_q(o[3, 4].astype(np.float64), light, a, b) for (a, b) in CORNERS]
    assert max(qs) / min(qs) > 2.0
    assert 0.1 < min(refs.values()) and max(refs.values()) < 0.9 * max(1.0, max(refs.values()))
    return mode, sc, gb, refs, light


def test_no_reuse_converges(low_light):
    mode, sc, gb, refs, light = low_light
    z = _z_scores(sc, gb, oracle.params(mode, "none", light=light, seed=7), refs)
    assert np.abs(z).max() < Z_MAX, z


@pytest.mark.parametrize("pattern,size", [("window", 2), ("group", 8)])
def test_unbiased_converges(low_light, pattern, size):
    mode, sc, gb, refs, light = low_light
    z = _z_scores(sc, gb, oracle.params(mode, "unbiased", pattern, radius=size, group_n=size, light=light, seed=7),
                  refs)
    assert np.abs(z).max() < Z_MAX, z
