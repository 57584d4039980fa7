"""Pins of the oracle's simple reuse baselines of Sec. 6: final-value
filtering (Filter (N); for shadows Light (N), light-sample reuse without
validation, which the paper notes reduces to the same average) and
light-sample reuse with visibility re-evaluation (Light (NU)).

Single-pixel sets reduce both to the no-reuse estimator; Light (NU) is
unbiased, so its mean converges to an FP64 quadrature of the shadow; the mean
of Filter (N) converges to the average of the true values over the set (its
bias is spatial blur), checked against per-pixel quadratures."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w

M = 4096
Z_MAX = 4.0
SIGMA_REF = 1e-3


def _oscene(parts):
    s = scenes.build([scenes.FLOOR] + parts)
    return oracle.Scene(s.V, s.F, grid=True)


def _light():
    return w.RectLight(np.array([0.0, 2.0, 0.0], np.float32), np.array([1.0, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, 1.0], np.float32))


def _shadow_case(tilted):
    sc = _oscene([scenes.plate_y(1.0, -0.5, 0.02, -3, 3), scenes.plate_y(0.1, -0.12, -0.06, -3, 3)])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    if tilted:
        th = np.arctan2(1.0, -0.1)
        gb.nrm[:] = np.array([np.sin(th), np.cos(th), 0.0], np.float32)
    return sc, gb


@pytest.mark.parametrize("mode", ["ao", "shadow"])
def test_single_pixel_filter_is_no_reuse(mode):
    sc, gb = _shadow_case(False)
    light = _light() if mode == "shadow" else None
    _, r0 = oracle.frame(sc, gb, oracle.params(mode, "none", light=light, ao_radius=1.0, seed=4))
    _, r1 = oracle.frame(sc, gb, oracle.params(mode, "filter", "group", group_n=1, light=light, ao_radius=1.0,
                                               seed=4))
    assert np.array_equal(r1.value, r0.value)


@pytest.mark.parametrize("tilted", [False, True])
def test_single_pixel_light_reuse_is_no_reuse(tilted):
    # the target re-traces its own light sample: the same decision as its trace
    sc, gb = _shadow_case(tilted)
    light = _light()
    for seed in (1, 2, 3):
        _, r0 = oracle.frame(sc, gb, oracle.params("shadow", "none", light=light, seed=seed))
        _, r1 = oracle.frame(sc, gb, oracle.params("shadow", "light", "group", group_n=1, light=light, seed=seed))
        ok = r1.nvar == 1
        assert ok.mean() > 0.95
        assert np.array_equal(r1.value[ok], r0.value[ok])


def test_filter_of_an_open_plane_is_one():
    sc = _oscene([])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    for mode in ("ao", "shadow"):
        _, r = oracle.frame(sc, gb, oracle.params(mode, "filter", "window", radius=2, light=_light(),
                                                  ao_radius=1.0, seed=2))
        assert np.all(r.value == 1.0)
    _, r = oracle.frame(sc, gb, oracle.params("shadow", "light", "window", radius=2, light=_light(), seed=2))
    assert np.all(r.value == 1.0)


TARGETS = [(x, y) for y in (3, 4) for x in (4, 5, 6, 7)]


def _mean_z(sc, gb, p, refs):
    s, s2 = oracle.render(sc, gb, p, M, region=(4, 3, 8, 5))
    zs = []
    for (x, y) in TARGETS:
        m = s[y, x] / M
        var = max(s2[y, x] / M - m * m, 0.0)
        zs.append((m - refs[(x, y)]) / np.sqrt(var / M + SIGMA_REF ** 2))
    return np.array(zs)


@pytest.mark.parametrize("tilted", [False, True])
@pytest.mark.parametrize("pattern,size", [("window", 1), ("window", 3), ("group", 8)])
def test_light_reuse_is_unbiased(tilted, pattern, size):
    sc, gb = _shadow_case(tilted)
    light = _light()
    o, _, _ = oracle.samples(gb, oracle.params("shadow", "none", light=light))
    refs = {(x, y): sc.shadow_quadrature(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), light,
                                         ign=0, ngrid=1024) for (x, y) in TARGETS}
    z = _mean_z(sc, gb, oracle.params("shadow", "light", pattern, radius=size, group_n=size, light=light,
                                      seed=11), refs)
    assert np.abs(z).max() < Z_MAX, z


def test_filter_converges_to_the_window_average():
    # E[Filter_i] = mean over S(i) of the true AO values (a blur, not the
    # value at i): checked against per-pixel quadratures, and the test has
    # the power to tell it from the pixel's own value
    sc = _oscene([scenes.plate_y(0.12, -3, 0, -3, 3), scenes.wall_x(0.3, 0, 3, -3, 3)])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    o, _, _ = oracle.samples(gb, oracle.params("ao", "none"))
    q = {}
    for y in range(2, 6):
        for x in range(3, 9):
            q[(x, y)] = sc.ao_quadrature(o[y, x].astype(np.float64), [0, 1, 0], 1.0, ign=0, nstrata=768)
    refs = {(x, y): np.mean([q[(x + dx, y + dy)] for dy in (-1, 0, 1) for dx in (-1, 0, 1)]) for (x, y) in TARGETS}
    p = oracle.params("ao", "filter", "window", radius=1, ao_radius=1.0, seed=5)
    z = _mean_z(sc, gb, p, refs)
    assert np.abs(z).max() < Z_MAX, z
    zself = _mean_z(sc, gb, p, {t: q[t] for t in TARGETS})
    assert np.abs(zself).max() > 6.0, zself
