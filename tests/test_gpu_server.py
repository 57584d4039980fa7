"""Served loop on the GPU: requests over resident scenes run concurrently on
stream slots under an HBM budget.  Every result must be bitwise identical to
the same request run alone through the per-view entry points, whether it ran
in a mix with overlapping requests, waited for memory, or wrote to a
server-held output.  The mix holds AO, shadows, solid-angle shadows and
direct illumination, with lights sampled uniformly or from the bilinear
density."""
import time

import numpy as np
import pytest

import oracle
import workloads as w
from gpu_util import compare_hits, compare_values, log, mismatch_reach, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


BOX_LIGHT = w.RectLight(np.array([0.0, 6.0, 0.0], np.float32), np.array([2.0, 0.0, 0.0], np.float32),
                        np.array([0.0, 0.0, 2.0], np.float32))
SIZES = [(160, 90), (96, 96), (257, 131)]
CONFIGS = [("window", 3, "biased"), ("window", 2, "unbiased"), ("group", 8, "biased"), ("window", 3, "none")]
DI_RADIANCE, DI_ALBEDO = 50.0, 0.7


@pytest.fixture(scope="module")
def world(ocr):
    scenes = [w.boxes_scene(1), w.terrain_scene(seed=10, cells=64, nspheres=20)]
    bvhs = [ocr.build_bvh(s.V, s.F) for s in scenes]
    pools = []
    for si, s in enumerate(scenes):
        pool = []
        for k, (W, H) in enumerate(SIZES):
            cam = w.boxes_camera(W, H) if si == 0 else w.orbit_camera(k, 3, W, H)
            gb = w.render_gbuffer(s, cam)
            pool.append((gb, ocr.DeviceGBuffer.from_host(gb)))
        pools.append(pool)
    lights = [BOX_LIGHT, w.terrain_light()]
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(24):
        si, vi = int(rng.integers(2)), int(rng.integers(len(SIZES)))
        mode = ["ao", "shadow", "shadow_sa", "di"][int(rng.integers(4))]
        pattern, size, est = CONFIGS[int(rng.integers(len(CONFIGS)))]
        light = None
        if mode != "ao":
            b = lights[si]
            light = w.RectLight(b.center, b.edge_u, b.edge_v, int(rng.integers(2)))  # either density
        reqs.append(dict(si=si, vi=vi, mode=mode, R=1.0 if si == 0 else 2.0, light=light, seed=1000 + i,
                         sample=i % 4, params=ocr.reuse_params(pattern, size, size, est)))
    # each request alone, through the per-view entry points
    for r in reqs:
        dg, bvh = pools[r["si"]][r["vi"]][1], bvhs[r["si"]]
        occ = ocr.trace_occluders(bvh, dg, "ao" if r["mode"] == "ao" else "shadow", r["R"], r["light"], r["seed"],
                                  r["sample"])
        if r["mode"] == "ao":
            out = ocr.reuse_ao(bvh, dg, occ, r["R"], r["params"])
        elif r["mode"] == "shadow":
            out = ocr.reuse_shadow(bvh, dg, occ, r["light"], r["params"])
        elif r["mode"] == "shadow_sa":
            out = ocr.reuse_shadow_solid_angle(bvh, dg, occ, r["light"], r["params"])
        else:
            out = ocr.reuse_direct_illumination(bvh, dg, occ, r["light"], r["params"], radiance=DI_RADIANCE,
                                                albedo=DI_ALBEDO)
        torch.cuda.synchronize()
        r["ref"] = to_np(out).copy()
    return bvhs, pools, reqs, scenes


def _serve(ocr, bvhs, pools, reqs, budget, slots, held, pace_ms=0.0):
    srv = ocr.Server(budget, slots=slots)
    sids = [srv.add_scene(bvhs[i], [dg for _, dg in pools[i]]) for i in range(2)]
    outs = {}
    tickets = {}
    bufs = [None if held else torch.full((SIZES[r["vi"]][1], SIZES[r["vi"]][0]), float("nan"), dtype=torch.float32,
                                         device="cuda") for r in reqs]
    # the server's streams do not wait on torch's: inputs and outputs must be ready
    torch.cuda.synchronize()
    for k, r in enumerate(reqs):
        out = bufs[k]
        rq = ocr.request(sids[r["si"]], r["vi"], r["mode"], r["R"], r["light"], r["seed"], r["sample"], r["params"],
                         out, radiance=DI_RADIANCE, albedo=DI_ALBEDO)
        t = srv.submit(rq)
        tickets[t] = k
        outs[t] = out
        if pace_ms:
            time.sleep(pace_ms * 1e-3)
    got = {}
    t0 = time.time()
    while len(got) < len(reqs):
        for res in srv.poll():
            assert res.status == 0, res.status
            k = tickets[res.ticket]
            W, H = SIZES[reqs[k]["vi"]]
            assert (res.width, res.height) == (W, H)
            if held:
                got[k] = ocr.device_to_host(res.out, (H, W), np.float32)
                srv.release(res.ticket)
            else:
                got[k] = None
        assert time.time() - t0 < 60, "server did not finish"
        time.sleep(0.001)
    torch.cuda.synchronize()
    for t, k in tickets.items():
        if not held:
            got[k] = to_np(outs[t])
    st = srv.stats()
    srv.destroy()
    return got, st


@pytest.mark.parametrize("held", [False, True])
def test_mix_equals_alone(ocr, world, held):
    bvhs, pools, reqs, _ = world
    log(f"[server] 24 requests, 6 slots, held={held}")
    got, st = _serve(ocr, bvhs, pools, reqs, 1 << 30, 6, held)
    for k, r in enumerate(reqs):
        assert np.array_equal(got[k].view(np.uint32), r["ref"].view(np.uint32)), k
    log(f"    max in flight {st.max_in_flight}, p50 {st.p50_ms:.3f} ms, p99 {st.p99_ms:.3f} ms")
    assert st.completed == len(reqs) and st.max_in_flight > 1


def test_budget_waits_and_still_equal(ocr, world):
    bvhs, pools, reqs, _ = world
    # room for one 257x131 request's records (28 B/px) at a time, or a few small ones
    W, H = SIZES[2]
    budget = int(28 * W * H * 1.2) + 4096
    log(f"[server] tight budget {budget} bytes")
    sub = [r for r in reqs if r["params"].estimator != 2]  # unbiased workspaces would not fit
    got, st = _serve(ocr, bvhs, pools, sub, budget, 6, False)
    for k, r in enumerate(sub):
        assert np.array_equal(got[k].view(np.uint32), r["ref"].view(np.uint32)), k
    assert st.waited_for_memory > 0 and st.peak_bytes <= budget


def test_refuses_oversized(ocr, world):
    bvhs, pools, reqs, _ = world
    srv = ocr.Server(1 << 16, slots=2)
    sid = srv.add_scene(bvhs[0], [dg for _, dg in pools[0]])
    st, _ = srv.try_submit(ocr.request(sid, 2, "ao", 1.0, out=None))
    assert st == -5
    srv.destroy()


def test_paced_arrivals_statistics(ocr, world):
    bvhs, pools, reqs, _ = world
    log("[server] paced arrivals")
    got, st = _serve(ocr, bvhs, pools, reqs, 1 << 30, 4, False, pace_ms=0.5)
    for k, r in enumerate(reqs):
        assert np.array_equal(got[k].view(np.uint32), r["ref"].view(np.uint32)), k
    assert 0 < st.p50_ms <= st.p99_ms <= st.max_ms
    assert st.frames_per_s > 0


@pytest.mark.parametrize("held", [False, True])
def test_mix_matches_oracle(ocr, world, held):
    # The accuracy bar of the served loop, checked against the oracle and not
    # only against the library's own per-view path: AO and shadow requests
    # (7x7 window, biased and unbiased) served in the middle of the 24-request
    # mix, with other requests in flight, each compared target by target
    # with the oracle's estimate of the same request.
    bvhs, pools, reqs, scenes = world
    checked = []
    for i, (mode, est) in enumerate([("ao", "biased"), ("ao", "unbiased"), ("shadow", "biased"),
                                     ("shadow", "unbiased")]):
        checked.append(dict(si=1, vi=2, mode=mode, R=2.0, light=w.terrain_light() if mode == "shadow" else None,
                            seed=5000 + i, sample=1, est=est, params=ocr.reuse_params("window", 3, 3, est)))
    mix = reqs[:12] + checked + reqs[12:]
    log(f"[server vs oracle] {len(mix)} requests, 6 slots, held={held}")
    got, st = _serve(ocr, bvhs, pools, mix, 1 << 30, 6, held)
    assert st.completed == len(mix) and st.max_in_flight > 1
    osc = oracle.Scene(scenes[1].V, scenes[1].F)
    gb, dg = pools[1][2]
    for c in checked:
        k = next(i for i, r in enumerate(mix) if r is c)
        # the request's records, traced alone (records are a pure function
        # of the inputs and the seed), name the rays whose hits differ
        occ = ocr.trace_occluders(bvhs[1], dg, c["mode"], c["R"], c["light"], c["seed"], c["sample"])
        torch.cuda.synchronize()
        p = oracle.params(c["mode"], c["est"], "window", radius=3, ao_radius=c["R"], light=c["light"],
                          seed=c["seed"], sample=c["sample"])
        rec, res = oracle.frame(osc, gb, p)
        gh = occ.hit_u32()
        hs = compare_hits(gh, rec, gb.valid)
        vs = compare_values(got[k], res, exclude=mismatch_reach(gh, rec, p))
        log(f"    {c['mode']} {c['est']}: hits {hs}; values {vs}")
        assert vs["compared"] > 0.99 * vs["targets"]
