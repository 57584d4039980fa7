"""Pins of the oracle's first-hit tracer (the predicate of Sec. 4.2 Eq.
occ-first-hit and the closest-hit queries of App. D / App. H): hand-built
rays with known answers, watertightness on closed fans, and the uniform-grid
candidate sets against plain brute force."""
import numpy as np
import pytest

import oracle
import workloads as w

MISS = oracle.MISS


def _tri_scene(tris):
    V = np.asarray(tris, np.float32).reshape(-1, 3)
    F = np.arange(V.shape[0], dtype=np.uint32).reshape(-1, 3)
    return oracle.Scene(V, F, grid=False), oracle.Scene(V, F, grid=True)


@pytest.mark.parametrize("grid", [False, True])
def test_hand_built_rays(grid):
    sc = _tri_scene([[(0, 0, 5), (2, 0, 5), (0, 2, 5)],        # 0: plane z=5
                     [(0, 0, 3), (2, 0, 3), (0, 2, 3)],        # 1: plane z=3 (closer)
                     [(10, 10, 1), (12, 10, 1), (10, 12, 1)]])[int(grid)]
    o = np.array([[0.5, 0.5, 0.0]])
    up = np.array([[0.0, 0.0, 1.0]])
    tri, t, g = sc.closest(o, up, 10.0)
    assert tri[0] == 1 and abs(t[0] - 3.0) < 1e-12 and not g[0]
    # ignoring the closer one reveals the farther one
    tri, t, g = sc.closest(o, up, 10.0, ign0=1)
    assert tri[0] == 0 and abs(t[0] - 5.0) < 1e-12
    # t_max between the two planes, inclusive end point
    tri, t, g = sc.closest(o, up, 3.0, inclusive=True)
    assert tri[0] == 1 and g[0]          # hit exactly at t_max: grazing
    tri, t, g = sc.closest(o, up, 2.9)
    assert tri[0] == MISS and not g[0]
    # behind the origin
    tri, t, g = sc.closest(o, -up, 10.0)
    assert tri[0] == MISS and not g[0]
    # outside the triangle
    tri, t, g = sc.closest([[1.5, 1.5, 0.0]], up, 10.0)
    assert tri[0] == MISS and not g[0]
    # parallel to the planes
    tri, t, g = sc.closest([[0.5, 0.5, 3.0 - 1e-3]], [[1.0, 0.0, 0.0]], 10.0)
    assert tri[0] == MISS
    # through an edge (x + y = 2 is the hypotenuse) -> flagged grazing
    tri, t, g = sc.closest([[1.0, 1.0, 0.0]], up, 10.0)
    assert g[0]
    # any-hit agrees with closest
    b, g = sc.any_hit(o, up, 10.0)
    assert b[0] and not g[0]
    b, g = sc.any_hit(o, up, 2.0)
    assert not b[0] and not g[0]
    b, g = sc.any_hit(o, up, 10.0, ign0=0, ign1=1)
    assert not b[0]


def test_tie_break_and_coplanar_duplicates():
    a = [(0, 0, 2), (4, 0, 2), (0, 4, 2)]
    sc = _tri_scene([a, a])[0]
    tri, t, g = sc.closest([[0.5, 0.5, 0.0]], [[0.0, 0.0, 1.0]], 10.0)
    assert tri[0] == 0  # equal t: smaller id
    assert g[0]         # and flagged: the FP32 kernel may pick either


def test_closed_fan_is_watertight():
    # rays aimed at the shared centre vertex and at points on shared edges of
    # a closed triangle fan must never pass through: every one either hits a
    # triangle or is flagged as grazing (and it hits in FP64 as well).
    rng = np.random.default_rng(0)
    m = 12
    ang = np.sort(rng.uniform(0, 2 * np.pi, m))
    ring = np.stack([np.cos(ang) * 2, np.sin(ang) * 2, np.full(m, 4.0)], 1)
    centre = np.array([0.1, -0.2, 4.0])
    tris = [[centre, ring[i], ring[(i + 1) % m]] for i in range(m)]
    sc = _tri_scene(tris)[0]
    origins = rng.uniform(-1, 1, (400, 3)) * [3, 3, 0]
    targets = [centre] + [centre + (ring[i] - centre) * f for i in range(m) for f in (0.25, 0.5, 0.9)]
    for tgt in targets:
        d = tgt - origins
        tri, t, g = sc.closest(origins, d, 2.0)
        assert (tri != MISS).all()
        assert g.all()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_grid_equals_brute_force_random_soup(seed):
    rng = np.random.default_rng(seed)
    n = 600
    c = rng.uniform(-5, 5, (n, 1, 3))
    tris = c + rng.normal(0, 0.6, (n, 3, 3))
    V = tris.reshape(-1, 3).astype(np.float32)
    F = np.arange(V.shape[0], dtype=np.uint32).reshape(-1, 3)
    sb = oracle.Scene(V, F, grid=False)
    sg = oracle.Scene(V, F, grid=True)
    assert oracle._load().orc_scene_grid_cells(sg.h) > 1
    o = rng.uniform(-6, 6, (4000, 3))
    d = rng.normal(0, 1, (4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tmax = rng.uniform(0.1, 15, 4000)
    ign = rng.integers(0, n, 4000).astype(np.uint32)
    r1 = sb.closest(o, d, tmax, ign0=ign)
    r2 = sg.closest(o, d, tmax, ign0=ign)
    assert np.array_equal(r1[0], r2[0])
    assert np.array_equal(r1[1], r2[1])
    assert np.array_equal(r1[2], r2[2])
    assert (r1[0] != MISS).mean() > 0.2
    a1 = sb.any_hit(o, d, tmax, ign0=ign)
    a2 = sg.any_hit(o, d, tmax, ign0=ign)
    assert np.array_equal(a1[0], a2[0])
    # any-hit is the closest hit's existence (exclusive end point)
    r3 = sb.closest(o, d, tmax, inclusive=False, ign0=ign)
    ok = ~a1[1] & ~r3[2]
    assert np.array_equal(a1[0][ok], (r3[0] != MISS)[ok])


def test_grid_equals_brute_force_on_boxes_scene():
    s = w.boxes_scene(1)
    gb = w.render_gbuffer(s, w.boxes_camera(96, 96))
    sb = oracle.Scene(s.V, s.F, grid=False)
    sg = oracle.Scene(s.V, s.F, grid=True)
    p = oracle.params("ao", "none", ao_radius=1.0, seed=3)
    r1 = oracle.records(sb, gb, p)
    r2 = oracle.records(sg, gb, p)
    assert np.array_equal(r1.hit, r2.hit)
    assert np.array_equal(r1.z, r2.z)
    assert np.array_equal(r1.graze, r2.graze)
    assert (r1.hit[gb.valid] != MISS).mean() > 0.02


def test_records_geometry():
    # hit point lies on the ray at the reported distance; oriented normal faces the origin
    s = w.boxes_scene(1)
    gb = w.render_gbuffer(s, w.boxes_camera(64, 64))
    sc = oracle.Scene(s.V, s.F)
    p = oracle.params("ao", "none", ao_radius=1.0, seed=5)
    rec = oracle.records(sc, gb, p)
    o, d, kind = oracle.samples(gb, p)
    hit = rec.hit != MISS
    assert hit.sum() > 10
    w_ = rec.z[hit] - o[hit].astype(np.float64)
    dd = d[hit].astype(np.float64)
    cross = np.cross(w_, dd)
    assert np.abs(cross).max() < 1e-9
    assert (np.einsum("ij,ij->i", rec.nz[hit], dd) < 0).all()
    assert (np.linalg.norm(w_, axis=1) <= 1.0 * np.linalg.norm(dd, axis=1) + 1e-12).all()
    assert np.allclose(np.linalg.norm(rec.nz[hit], axis=1), 1.0)
