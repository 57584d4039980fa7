"""GPU tracing robustness against the oracle's brute force (the first-hit
predicate of Sec. 4.2 Eq. occ-first-hit; step 1 of App. D / App. H):

* closed triangle fans: shadow segments aimed through the shared centre
  vertex and through points of the shared edges must never slip between the
  triangles (watertightness), and must hit a triangle that holds the aimed
  point;
* random triangle soups: 10^5 AO rays and shadow segments from receivers
  scattered inside the soup, hit ids against the oracle's brute force (only
  rays the oracle flags as grazing may differ, at most 1e-5 of them).

The receivers are hand-placed G-buffer entries (position, normal, an id of
a far-away triangle so that nothing in the soup or fan is ignored)."""
import math

import numpy as np
import pytest

import oracle
import workloads as w
from gpu_util import compare_hits, compare_records, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


FAR = [(1000.0, 1000.0, 1000.0), (1001.0, 1000.0, 1000.0), (1000.0, 1001.0, 1000.0)]


def _scene(tris):
    """Triangles as given, then one far-away triangle (the receivers' own id)."""
    V = np.asarray(list(tris) + [FAR], np.float64).reshape(-1, 3).astype(np.float32)
    F = np.arange(V.shape[0], dtype=np.uint32).reshape(-1, 3)
    return w.Scene(V, F), F.shape[0] - 1


def _gbuffer(pos, nrm, own):
    n = pos.shape[0]
    W = 256
    H = -(-n // W)
    P = np.zeros((H * W, 3), np.float32)
    N = np.zeros((H * W, 3), np.float32)
    prim = np.full(H * W, 0xFFFFFFFF, np.uint32)
    P[:n] = pos
    N[:n] = nrm
    prim[:n] = own
    return w.GBuffer(P.reshape(H, W, 3), N.reshape(H, W, 3), prim.reshape(H, W))


def _fan(rng, m, centre, radius, z):
    ang = np.sort(rng.uniform(0, 2 * np.pi, m))
    ring = np.stack([np.cos(ang) * radius, np.sin(ang) * radius, np.full(m, z)], 1)
    tris = [[centre, ring[i], ring[(i + 1) % m]] for i in range(m)]
    return tris, ring


@pytest.mark.parametrize("seed,m", [(0, 12), (1, 64), (2, 5)])
def test_closed_fan_segments_never_leak(ocr, seed, m):
    rng = np.random.default_rng(seed)
    centre = np.array([0.1, -0.2, 4.0])
    tris, ring = _fan(rng, m, centre, 2.0, 4.0)
    scene, own = _scene(tris)
    bvh = ocr.build_bvh(scene.V, scene.F)
    # a light 1e-5 m across, 4 m above the fan; each receiver sits on the line
    # from the light's centre through an aimed point (the centre vertex, or a
    # point of a shared edge), below the fan, with its normal towards the light
    c = np.array([0.3, 0.1, 8.0])
    # (e_u x e_v = -z: the light emits downwards, towards the receivers)
    light = w.RectLight(c.astype(np.float32), np.array([0, 1e-5, 0], np.float32), np.array([1e-5, 0, 0], np.float32))
    aims, owners = [centre], [set(range(m))]
    for i in range(m):
        for f in (0.25, 0.5, 0.9):
            aims.append(centre + (ring[i] - centre) * f)
            owners.append({(i - 1) % m, i})  # triangles i-1 and i share the edge to ring[i]
    pos, nrm, which = [], [], []
    for a_i, a in enumerate(aims):
        lam = rng.uniform(0.05, 2.0, 400)
        x = a[None, :] + (a - c)[None, :] * lam[:, None]
        x += rng.normal(0, 1e-9, x.shape)
        d = c[None, :] - x
        pos.append(x)
        nrm.append(d / np.linalg.norm(d, axis=1, keepdims=True))
        which.append(np.full(lam.size, a_i))
    pos, nrm, which = np.concatenate(pos), np.concatenate(nrm), np.concatenate(which)
    gb = _gbuffer(pos, nrm, own)
    dg = ocr.DeviceGBuffer.from_host(gb)
    log(f"[fan] m={m}: {len(aims)} aimed points, {pos.shape[0]} segments")
    hits = []
    for sample in range(4):
        occ = ocr.trace_occluders(bvh, dg, "shadow", 1.0, light, seed=seed + 1, sample=sample)
        torch.cuda.synchronize()
        h = occ.hit_u32().ravel()[:pos.shape[0]]
        assert (h != oracle.SELF).all()
        leak = h == oracle.MISS
        assert not leak.any(), f"{int(leak.sum())} segments slipped through (aims {sorted(set(which[leak]))[:8]})"
        ok = np.array([int(hh) in owners[a_i] for hh, a_i in zip(h, which)])
        assert ok.all(), "a segment hit a triangle that does not hold its aimed point"
        hits.append(h)
        # the oracle sees no leak either
        osc = oracle.Scene(scene.V, scene.F, grid=False)
        rec = oracle.records(osc, gb, oracle.params("shadow", "none", light=light, seed=seed + 1, sample=sample))
        assert (rec.hit.ravel()[:pos.shape[0]] != oracle.MISS).all()
    # the fans' hits spread over the triangles around the aimed points
    assert len(set(np.concatenate(hits).tolist())) >= min(m, 5)


def _soup(rng, n, spread):
    c = rng.uniform(-5, 5, (n, 1, 3))
    return (c + rng.normal(0, spread, (n, 3, 3))).tolist()


@pytest.mark.parametrize("seed", [0, 1])
def test_random_soup_hits_match_brute_force(ocr, seed):
    rng = np.random.default_rng(100 + seed)
    scene, own = _scene(_soup(rng, 800, 0.6))
    bvh = ocr.build_bvh(scene.V, scene.F)
    n = 100_000
    pos = rng.uniform(-6, 6, (n, 3))
    nrm = rng.normal(0, 1, (n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    gb = _gbuffer(pos, nrm, own)
    dg = ocr.DeviceGBuffer.from_host(gb)
    osc = oracle.Scene(scene.V, scene.F, grid=False)
    light = w.RectLight(np.array([0.0, 0.0, 9.0], np.float32), np.array([6.0, 0, 0], np.float32),
                        np.array([0, -6.0, 0], np.float32))
    for mode, R in (("ao", 3.0), ("ao", 12.0), ("shadow", 1.0)):
        log(f"[soup {seed}] {mode} R={R}: {n} rays over {scene.ntris} triangles")
        occ = ocr.trace_occluders(bvh, dg, mode, R, light if mode == "shadow" else None, seed=7 + seed)
        torch.cuda.synchronize()
        p = oracle.params(mode, "none", ao_radius=R, light=light if mode == "shadow" else None, seed=7 + seed)
        rec = oracle.records(osc, gb, p)
        gh = occ.hit_u32()
        st = compare_hits(gh, rec, gb.valid)
        o, _, _ = oracle.samples(gb, p)
        nrec = compare_records(occ.dz.cpu().numpy(), occ.nz.cpu().numpy(), gh, rec, o, scene)
        log(f"    {st}, records compared {nrec}")
        assert st["rays"] > 0.4 * n and nrec > 0.1 * st["rays"]
        assert st["mismatches"] <= math.ceil(1e-5 * st["rays"])
