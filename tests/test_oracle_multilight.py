"""Pins of the oracle's shadows of several rectangular lights.  The paper
shows a two-light result without a formulation; the reading taken: the
visible fraction of the total emitting area, sum_l (A_l / A_tot) Shadow_l,
with each sample on light l with probability A_l / A_tot (uniform over the
union), the induced density summed over the lights and F_i their
area-weighted front fraction.

A one-element list is the single light; coincident copies of one light give
exactly its estimate (the combination weights); the light choice follows the
area ratio; no-reuse and unbiased estimates converge to the area-weighted sum
of per-light FP64 quadratures."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w


def _light(cx=0.0, Hl=2.0, L=1.0, cz=0.0):
    return w.RectLight(np.array([cx, Hl, cz], np.float32), np.array([L, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, L], np.float32))


def _case():
    s = scenes.build([scenes.FLOOR, scenes.plate_y(1.0, -0.5, 0.02, -3, 3), scenes.plate_y(0.1, -0.12, -0.06, -3, 3)])
    return oracle.Scene(s.V, s.F, grid=True), scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)


@pytest.mark.parametrize("est", ["none", "biased", "unbiased"])
def test_one_light_list_is_the_single_light(est):
    sc, gb = _case()
    a = oracle.frame(sc, gb, oracle.params("shadow", est, "window", radius=2, light=_light(), seed=3))
    b = oracle.frame(sc, gb, oracle.params("shadow", est, "window", radius=2, light=[_light()], seed=3))
    assert np.array_equal(a[0].hit, b[0].hit)
    assert np.array_equal(a[1].value, b[1].value)


@pytest.mark.parametrize("est", ["none", "biased", "unbiased"])
def test_coincident_copies_are_one_light(est):
    sc, gb = _case()
    for seed in (1, 2):
        a = oracle.frame(sc, gb, oracle.params("shadow", est, "window", radius=2, light=_light(), seed=seed))
        b = oracle.frame(sc, gb, oracle.params("shadow", est, "window", radius=2, light=[_light(), _light()],
                                               seed=seed))
        assert np.array_equal(a[0].hit, b[0].hit)
        np.testing.assert_allclose(b[1].value, a[1].value, rtol=1e-12, atol=1e-15)


def test_light_choice_follows_the_area_ratio():
    # lights of areas 1 and 4 far apart: a sample's point tells its light
    gb = scenes.floor_grid(64, 64, 0.01, x0=-0.3, z0=-0.3)
    la, lb = _light(cx=-3.0, L=1.0), _light(cx=3.0, L=2.0)
    n, hits_b = 0, 0
    for s in range(8):
        o, d, kind = oracle.samples(gb, oracle.params("shadow", "none", light=[la, lb], seed=9, sample=s))
        y = o + d
        ok = kind < 2
        n += int(ok.sum())
        hits_b += int(((y[..., 0] > 0) & ok).sum())
    frac = hits_b / n
    assert abs(frac - 0.8) < 4 * np.sqrt(0.8 * 0.2 / n)


TARGETS = [(x, y) for y in (3, 4) for x in (4, 5, 6, 7)]
M = 4096


def _z(sc, gb, p, refs):
    s, s2 = oracle.render(sc, gb, p, M, region=(4, 3, 8, 5))
    out = []
    for (x, y) in TARGETS:
        m = s[y, x] / M
        var = max(s2[y, x] / M - m * m, 0.0)
        out.append((m - refs[(x, y)]) / np.sqrt(var / M + 1e-6))
    return np.array(out)


@pytest.fixture(scope="module")
def two_lights():
    sc, gb = _case()
    lights = [_light(cx=-0.4, L=0.8), _light(cx=0.6, Hl=2.5, L=1.2)]
    areas = np.array([0.8 ** 2, 1.2 ** 2])
    wts = areas / areas.sum()
    o, _, _ = oracle.samples(gb, oracle.params("shadow", "none", light=lights))
    refs = {}
    for (x, y) in TARGETS:
        q = [sc.shadow_quadrature(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), lt, ign=0,
                                  ngrid=768) for lt in lights]
        refs[(x, y)] = float(wts @ np.array(q))
    return sc, gb, lights, refs


def test_two_lights_no_reuse_converges(two_lights):
    sc, gb, lights, refs = two_lights
    z = _z(sc, gb, oracle.params("shadow", "none", light=lights, seed=7), refs)
    assert np.abs(z).max() < 4.0, z


@pytest.mark.parametrize("pattern,size", [("window", 1), ("window", 3), ("group", 8)])
def test_two_lights_unbiased_converges(two_lights, pattern, size):
    sc, gb, lights, refs = two_lights
    z = _z(sc, gb, oracle.params("shadow", "unbiased", pattern, radius=size, group_n=size, light=lights, seed=7),
           refs)
    assert np.abs(z).max() < 4.0, z
