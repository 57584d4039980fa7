"""Pins of the oracle's reuse estimators (Sec. 4.2 Eqs. generic-mis-weight,
generic-mis-estimator-simplified; Sec. 4.3 Eqs. ao-unbiased-estimator,
ao-biased-estimator; Sec. 4.4 Eqs. shadow-estimator,
shadow-biased-estimator and the dark-region guard; App. D and App. H):
special cases that reduce to simpler estimators, the consistent-occluder
case where biased and unbiased coincide, the four reuse cases of the
shadow-reuse figure, and the statistical unbiasedness of the unbiased
estimator against FP64 quadrature (with a power check on the biased one)."""
import numpy as np
import pytest

import oracle
import scenes
import workloads as w

MISS = oracle.MISS


def _oscene(parts):
    s = scenes.build([scenes.FLOOR] + parts)
    return oracle.Scene(s.V, s.F, grid=True)


def _light(Hl=2.0, L=1.0, cx=0.0, cz=0.0):
    return w.RectLight(np.array([cx, Hl, cz], np.float32), np.array([L, 0.0, 0.0], np.float32),
                       np.array([0.0, 0.0, L], np.float32))


# --------------------------------------------------------------------------
# Reductions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("pattern,size", [("window", 0), ("group", 1)])
def test_single_pixel_set_reduces_to_no_reuse_ao(pattern, size):
    # S(i) = {i}: B_i = p_i(i) / p_i(i) = 1 for a hit, so 1 - B_i = 1 - [hit].
    s = w.boxes_scene(1)
    gb = w.render_gbuffer(s, w.boxes_camera(128, 128))
    sc = oracle.Scene(s.V, s.F)
    base = oracle.params("ao", "none", ao_radius=1.0, seed=3)
    rec0, r0 = oracle.frame(sc, gb, base)
    for est in ("biased", "unbiased"):
        p = oracle.params("ao", est, pattern, radius=size, group_n=size, ao_radius=1.0, seed=3)
        rec, r = oracle.frame(sc, gb, p)
        ok = gb.valid & (r.nvar == 1)
        assert ok.sum() > 0.95 * gb.valid.sum()
        assert np.array_equal(r.value[ok], r0.value[ok])
        assert (rec.hit[gb.valid] != MISS).any()


def test_single_pixel_set_reduces_to_no_reuse_shadow():
    # With the whole light in front of every receiver (F_i = 1), S(i) = {i}
    # gives 1 - [blocked], the no-reuse shadow estimator.
    sc = _oscene([scenes.plate_y(1.0, -0.3, 0.1, -0.2, 0.3)])
    gb = scenes.floor_grid(24, 16, 0.04, x0=-0.5, z0=-0.3)
    light = _light()
    p0 = oracle.params("shadow", "none", light=light, seed=2)
    _, r0 = oracle.frame(sc, gb, p0)
    p1 = oracle.params("shadow", "unbiased", "group", group_n=1, light=light, seed=2)
    _, r1 = oracle.frame(sc, gb, p1)
    ok = r1.nvar == 1
    assert ok.mean() > 0.95
    assert np.allclose(r1.value[ok], r0.value[ok], atol=1e-12)
    assert 0.1 < r0.value.mean() < 0.9


def test_identical_receivers_average_their_samples():
    # When every receiver of S(i) is the same point with the same normal, all
    # techniques share one density, the balance weights are 1/|S(i)| and the
    # MIS estimate is the plain average of the |S(i)| no-reuse estimates.
    sc = _oscene([scenes.wall_x(0.2, 0, 2, -2, 2), scenes.plate_y(0.7, -1, 1, -1, 1)])
    gb = scenes.floor_grid(9, 9, 0.0)
    base = oracle.params("ao", "none", ao_radius=1.0, seed=5)
    _, r0 = oracle.frame(sc, gb, base)
    for est in ("biased", "unbiased"):
        p = oracle.params("ao", est, "window", radius=2, ao_radius=1.0, seed=5)
        _, r = oracle.frame(sc, gb, p)
        for y in range(9):
            for x in range(9):
                ys, xs = slice(max(y - 2, 0), y + 3), slice(max(x - 2, 0), x + 3)
                assert r.value[y, x] == pytest.approx(r0.value[ys, xs].mean(), abs=1e-12)
    assert 0.2 < r0.value.mean() < 0.8


# --------------------------------------------------------------------------
# Consistent occluders: biased == unbiased (Sec. 4.3, local first-hit
# consistency holds exactly)
# --------------------------------------------------------------------------
def test_consistent_scene_biased_equals_unbiased():
    ao = _oscene([scenes.wall_x(0.35, 0, 3, -3, 3)])
    gb = scenes.floor_grid(16, 12, 0.04, x0=-0.3, z0=-0.2)
    for pattern, size in [("window", 2), ("window", 3), ("group", 8)]:
        pb = oracle.params("ao", "biased", pattern, radius=size, group_n=size, ao_radius=1.0, seed=9)
        pu = oracle.params("ao", "unbiased", pattern, radius=size, group_n=size, ao_radius=1.0, seed=9)
        _, rb = oracle.frame(ao, gb, pb)
        _, ru = oracle.frame(ao, gb, pu)
        assert np.array_equal(rb.value, ru.value)
        assert (rb.value < 1).mean() > 0.3
    sh = _oscene([scenes.plate_y(1.0, -0.2, 0.15, -3, 3)])
    for pattern, size in [("window", 3), ("group", 4)]:
        pb = oracle.params("shadow", "biased", pattern, radius=size, group_n=size, light=_light(), seed=9,
                           dark_guard=False)
        pu = oracle.params("shadow", "unbiased", pattern, radius=size, group_n=size, light=_light(), seed=9)
        _, rb = oracle.frame(sh, gb, pb)
        _, ru = oracle.frame(sh, gb, pu)
        assert np.array_equal(rb.value, ru.value)


# --------------------------------------------------------------------------
# The four reuse cases of the shadow-reuse figure (Sec. 4.4)
# --------------------------------------------------------------------------
def test_shadow_reuse_cases():
    light = _light(Hl=2.0, L=1.0)
    up = np.array([0.0, 1.0, 0.0])
    down = np.array([0.0, -1.0, 0.0])
    x1 = np.array([0.0, 0.0, 0.0])
    # (a) valid reuse: the ray from x1 through z2 meets the emitter -> density > 0
    z2 = np.array([0.1, 1.0, 0.0])
    assert oracle.density_shadow(x1, up, z2, down, light) > 0
    # J at y' : |x1 - y'|^2 / |x1 - z2|^2 = s^2 = 4, both cosines equal -> J = 4
    assert oracle.density_shadow(x1, up, z2, down, light) == pytest.approx(4.0, rel=1e-12)
    # (c) the ray from x1 through z2 misses the emitter (outside the rectangle)
    assert oracle.density_shadow(x1, up, np.array([0.4, 1.0, 0.0]), down, light) == 0.0
    # ... or the light lies in front of z (s < 1) -> chi = 0
    assert oracle.density_shadow(x1, up, np.array([0.05, 2.5, 0.0]), down, light) == 0.0
    # (b) and (d) at the estimator level: two receivers in one group of N=2
    # x1 at X=0 sits under a low strip; x2 at X=0.1 is not.  A high plate
    # blocks part of the light for both; x2's occluder on the high plate is
    # hidden from x1 by the strip, so its exact density at x1 is 0.
    sc = _oscene([scenes.plate_y(1.0, -1, 1, -1, 1), scenes.plate_y(0.05, -0.08, 0.06, -1, 1)])
    gb = scenes.floor_grid(2, 1, 0.1, x0=0.0, z0=0.0)
    pu = oracle.params("shadow", "unbiased", "group", group_n=2, light=light, seed=1)
    pb = oracle.params("shadow", "biased", "group", group_n=2, light=light, seed=1, dark_guard=False)
    rec = oracle.records(sc, gb, pu)
    assert (rec.hit != MISS).all()
    ru = oracle.reuse(sc, gb, pu, rec)
    rb = oracle.reuse(sc, gb, pb, rec)
    # x1's own candidate is on the strip; x2's is on the high plate:
    assert rec.z[0, 0, 1] == pytest.approx(0.05)
    assert rec.z[0, 1, 1] == pytest.approx(1.0)
    # unbiased: x2's candidate contributes nothing at x1 (case d), but the
    # biased estimator counts it
    assert ru.value[0, 0] != rb.value[0, 0]
    # (b) a missed source contributes nothing: a receiver whose ray misses
    # keeps B from that source at 0 -- move x2 out from under the plates
    gb2 = scenes.floor_grid(2, 1, 3.0, x0=0.0, z0=0.0)
    light2 = _light(Hl=2.0, L=0.2, cx=1.5)
    pb2 = oracle.params("shadow", "biased", "group", group_n=2, light=light2, seed=1, dark_guard=False)
    rec2 = oracle.records(_oscene([]), gb2, pb2)
    assert (rec2.hit == MISS).all()
    r2 = oracle.reuse(_oscene([]), gb2, pb2, rec2)
    assert np.allclose(r2.value, [[oracle.front_fraction([0, 0, 0], up, light2),
                                   oracle.front_fraction([3, 0, 0], up, light2)]])


def test_dark_guard():
    # Every sample of the set blocked -> the biased shadow estimate is 0.
    sc = _oscene([scenes.plate_y(1.0, -3, 3, -3, 3)])
    gb = scenes.floor_grid(12, 12, 0.05, x0=-0.3, z0=-0.3)
    light = _light()
    pg = oracle.params("shadow", "biased", "window", radius=2, light=light, seed=4, dark_guard=True)
    pn = oracle.params("shadow", "biased", "window", radius=2, light=light, seed=4, dark_guard=False)
    rec = oracle.records(sc, gb, pg)
    assert (rec.hit != MISS).all()
    rg = oracle.reuse(sc, gb, pg, rec)
    rn = oracle.reuse(sc, gb, pn, rec)
    assert (rg.value == 0.0).all()
    assert np.abs(rn.value).max() > 1e-3  # without the guard, F - B is not exactly 0
    # one unblocked sample in the set disables the guard for that target
    pu = oracle.params("shadow", "unbiased", "window", radius=2, light=light, seed=4)
    ru = oracle.reuse(sc, gb, pu, rec)
    assert np.allclose(ru.value, rn.value)  # consistent scene: biased (no guard) == unbiased


# --------------------------------------------------------------------------
# Unbiasedness (Sec. 6: unbiased reuse converges; App. J/K convergence plots)
# --------------------------------------------------------------------------
M = 4096
TARGETS = [(x, y) for y in (3, 4) for x in (4, 5, 6, 7)]
CONFIGS = [("window", 1), ("window", 2), ("window", 3), ("group", 2), ("group", 4), ("group", 8)]
SIGMA_REF = 1e-3  # quadrature error allowance
Z_MAX = 4.0       # family-wise ~1% over all pixels and configurations


def _z_scores(sc, gb, p, refs):
    s, s2 = oracle.render(sc, gb, p, M, region=(4, 3, 8, 5))
    zs = []
    for (x, y) in TARGETS:
        m = s[y, x] / M
        var = max(s2[y, x] / M - m * m, 0.0)
        zs.append((m - refs[(x, y)]) / np.sqrt(var / M + SIGMA_REF ** 2))
    return np.array(zs)


@pytest.fixture(scope="module")
def ao_inconsistent():
    # A low roof over X < 0 and a wall at X = 0.3: occluders that receivers
    # outside the roof find on the wall are hidden by the roof from receivers
    # under it, so first-hit consistency fails near the roof's edge.
    sc = _oscene([scenes.plate_y(0.12, -3, 0, -3, 3), scenes.wall_x(0.3, 0, 3, -3, 3)])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    o, _, _ = oracle.samples(gb, oracle.params("ao", "none"))
    refs = {(x, y): sc.ao_quadrature(o[y, x].astype(np.float64), [0, 1, 0], 1.0, ign=0, nstrata=1024)
            for (x, y) in TARGETS}
    return sc, gb, refs


@pytest.fixture(scope="module", params=["flat", "tilted"])
def shadow_inconsistent(request):
    # A high plate over X < 0.02 and a low strip over X in [-0.12, -0.06]:
    # high-plate occluders of outer receivers are hidden by the strip.
    light = _light()
    sc = _oscene([scenes.plate_y(1.0, -0.5, 0.02, -3, 3), scenes.plate_y(0.1, -0.12, -0.06, -3, 3)])
    gb = scenes.floor_grid(12, 8, 0.05, x0=-0.3, z0=-0.2)
    if request.param == "tilted":
        # tangent planes cut the light: F_i < 1
        th = np.arctan2(1.0, -0.1)
        gb.nrm[:] = np.array([np.sin(th), np.cos(th), 0.0], np.float32)
    o, _, _ = oracle.samples(gb, oracle.params("shadow", "none", light=light))
    refs = {(x, y): sc.shadow_quadrature(o[y, x].astype(np.float64), gb.nrm[y, x].astype(np.float64), light,
                                         ign=0, ngrid=1024) for (x, y) in TARGETS}
    return sc, gb, refs, light, request.param


def test_ao_no_reuse_converges(ao_inconsistent):
    sc, gb, refs = ao_inconsistent
    z = _z_scores(sc, gb, oracle.params("ao", "none", ao_radius=1.0, seed=7), refs)
    assert np.abs(z).max() < Z_MAX, z


@pytest.mark.parametrize("pattern,size", CONFIGS)
def test_ao_unbiased_converges_biased_does_not(ao_inconsistent, pattern, size):
    sc, gb, refs = ao_inconsistent
    pu = oracle.params("ao", "unbiased", pattern, radius=size, group_n=size, ao_radius=1.0, seed=7)
    zu = _z_scores(sc, gb, pu, refs)
    assert np.abs(zu).max() < Z_MAX, zu
    pb = oracle.params("ao", "biased", pattern, radius=size, group_n=size, ao_radius=1.0, seed=7)
    zb = _z_scores(sc, gb, pb, refs)
    assert np.abs(zb).max() > 6.0, zb  # power: the test detects the biased estimator's bias


@pytest.mark.parametrize("pattern,size", CONFIGS)
def test_shadow_unbiased_converges(shadow_inconsistent, pattern, size):
    sc, gb, refs, light, kind = shadow_inconsistent
    pu = oracle.params("shadow", "unbiased", pattern, radius=size, group_n=size, light=light, seed=7)
    zu = _z_scores(sc, gb, pu, refs)
    assert np.abs(zu).max() < Z_MAX, zu
    if kind == "flat":
        pb = oracle.params("shadow", "biased", pattern, radius=size, group_n=size, light=light, seed=7,
                           dark_guard=False)
        zb = _z_scores(sc, gb, pb, refs)
        assert np.abs(zb).max() > 6.0, zb


def test_shadow_no_reuse_converges(shadow_inconsistent):
    sc, gb, refs, light, kind = shadow_inconsistent
    z = _z_scores(sc, gb, oracle.params("shadow", "none", light=light, seed=7), refs)
    assert np.abs(z).max() < Z_MAX, z


# --------------------------------------------------------------------------
# Partition of unity of the balance heuristic
# --------------------------------------------------------------------------
@pytest.mark.parametrize("est", ["biased", "unbiased"])
@pytest.mark.parametrize("n", [2, 4, 8])
def test_group_weights_partition_unity(est, n):
    # Within a fixed group every target shares the denominators P(j), so
    # sum_{i in group} p_i(j) / P(j) = 1 for each candidate with P(j) > 0:
    # the group's B_i sum to its number of such candidates.  A hit whose own
    # density is positive has P(j) >= p_j(j) > 0, so on a scene where every
    # hit lies within R of its own receiver that is its number of hits.
    s = w.boxes_scene(1)
    gb = w.render_gbuffer(s, w.boxes_camera(64, 64))
    sc = oracle.Scene(s.V, s.F)
    p = oracle.params("ao", est, "group", group_n=n, ao_radius=1.0, seed=6)
    rec, r = oracle.frame(sc, gb, p)
    gw = 4 if n == 8 else (2 if n >= 2 else 1)
    gh = 2 if n >= 4 else 1
    H, W = gb.prim.shape
    checked = 0
    for y0 in range(0, H, gh):
        for x0 in range(0, W, gw):
            sl = (slice(y0, y0 + gh), slice(x0, x0 + gw))
            valid = gb.valid[sl]
            if not valid.any() or (r.nvar[sl][valid] != 1).any():
                continue
            B = (1.0 - r.value[sl][valid]).sum()
            hits = (rec.hit[sl][valid] < oracle.SELF).sum()
            assert B == pytest.approx(hits, abs=1e-9)
            checked += 1
    assert checked > 100
