"""Scheduling logic of the served loop, run without a device: the server's
mock executor makes no HIP call and lets each request occupy its slot for a
modelled time (mock_ns_per_pixel * w * h).  Covers FIFO admission, HBM-budget
waiting and refusal, overlap of requests in flight, queue limits, server-held
outputs, the latency statistics, and injected launch failures (the failing
request reports its error and gives back its memory; the server carries on)."""
import time

import numpy as np
import pytest

import paper_2607_23122_amd as ocr


def _server(budget, slots, ns_per_px=0.0, max_queue=0, fault_every=0):
    return ocr.Server(budget, slots=slots, max_queue=max_queue, poll_us=50, mock=True, mock_ns_per_pixel=ns_per_px,
                      fault_every=fault_every)


def _views(sizes):
    return [ocr._GBuffer(0, 0, 0, w, h) for (w, h) in sizes]


def _req(scene, view, mode="ao", out=1, **kw):
    light = np.array([0, 5, 0, 1, 0, 0, 0, 0, 1], np.float32) if mode == "shadow" else None
    return ocr.request(scene, view, mode=mode, ao_radius=1.0, light=light, out=out, **kw)


def _wait_done(srv, n, timeout=20.0):
    got = []
    t0 = time.time()
    while len(got) < n:
        got += srv.poll()
        if time.time() - t0 > timeout:
            raise AssertionError(f"only {len(got)} of {n} results after {timeout} s")
        time.sleep(0.002)
    return got


def test_fifo_one_slot():
    srv = _server(1 << 30, slots=1, ns_per_px=200.0)
    sid = srv.add_scene(None, _views([(64, 64)]))
    tickets = [srv.submit(_req(sid, 0, seed=i)) for i in range(6)]
    res = _wait_done(srv, 6)
    assert [r.ticket for r in res] == tickets
    for a, b in zip(res, res[1:]):
        assert b.start_ms >= a.end_ms - 1e-6  # one slot: strictly one after another
    st = srv.stats()
    assert st.completed == 6 and st.max_in_flight == 1 and st.queued == 0
    srv.destroy()


def test_slots_overlap():
    srv = _server(1 << 30, slots=4, ns_per_px=2000.0)  # 64x64 -> ~8 ms each
    sid = srv.add_scene(None, _views([(64, 64)]))
    for i in range(8):
        srv.submit(_req(sid, 0, seed=i))
    res = _wait_done(srv, 8)
    st = srv.stats()
    assert st.max_in_flight == 4
    # two waves of four: the fifth starts only after some first-wave request ended
    res.sort(key=lambda r: r.ticket)
    assert min(r.start_ms for r in res[4:]) >= min(r.end_ms for r in res[:4]) - 1e-6
    srv.destroy()


def test_budget_forces_waiting():
    w, h = 64, 64
    need = 2 * ((12 * w * h + 255) // 256 * 256) + (4 * w * h + 255) // 256 * 256  # records, caller-owned output
    srv = _server(need + need // 2, slots=4, ns_per_px=500.0)  # room for one request at a time
    sid = srv.add_scene(None, _views([(w, h)]))
    for i in range(5):
        srv.submit(_req(sid, 0, seed=i))
    res = _wait_done(srv, 5)
    st = srv.stats()
    assert st.max_in_flight == 1
    assert st.waited_for_memory > 0
    assert st.peak_bytes <= st.budget_bytes
    assert all(r.status == 0 for r in res)
    srv.destroy()


def test_refuses_what_never_fits_and_full_queue():
    srv = _server(1 << 20, slots=1, ns_per_px=1000.0, max_queue=2)
    sid = srv.add_scene(None, _views([(1920, 1080), (32, 32)]))
    st, _ = srv.try_submit(_req(sid, 0))
    assert st == -5  # OCR_ERR_BUDGET: 1080p records alone exceed 1 MiB
    assert b"budget" in ocr.lib().ocr_last_error()
    codes = [srv.try_submit(_req(sid, 1, seed=i))[0] for i in range(6)]
    # one may be admitted at once; the queue then holds two; the rest are refused as busy
    assert codes.count(0) >= 2 and -6 in codes
    assert srv.stats().refused == 1
    srv.drain()
    srv.destroy()


def test_argument_checks():
    srv = _server(1 << 30, slots=2)
    sid = srv.add_scene(None, _views([(16, 16)]))
    assert srv.try_submit(_req(sid + 1, 0))[0] == -1          # unknown scene
    assert srv.try_submit(_req(sid, 3))[0] == -1              # unknown view
    r = _req(sid, 0)
    r.mode = 7
    assert srv.try_submit(r)[0] == -1                        # bad mode
    r = _req(sid, 0)
    r.ao_radius = -1.0
    assert srv.try_submit(r)[0] == -1                        # bad radius
    r = _req(sid, 0, params=ocr.reuse_params("group", 0, 3, "biased"))
    assert srv.try_submit(r)[0] == -1                        # bad group size
    r = _req(sid, 0, params=ocr.reuse_params("window", 3, 0, "biased", accumulate=True))
    assert srv.try_submit(r)[0] == -1                        # accumulate not served
    bad_light = ocr.request(sid, 0, mode="shadow", light=np.zeros(9, np.float32), out=1)
    assert srv.try_submit(bad_light)[0] == -1                # degenerate light
    import workloads as w
    lt = w.RectLight(np.array([0, 5, 0], np.float32), np.array([1, 0, 0], np.float32),
                     np.array([0, 0, 1], np.float32), 1)
    for mode in ("shadow", "shadow_sa", "di"):
        assert srv.try_submit(ocr.request(sid, 0, mode=mode, light=lt, out=1))[0] == 0  # bilinear density served
    bad_di = ocr.request(sid, 0, mode="di", light=lt, out=1, radiance=-1.0)
    assert srv.try_submit(bad_di)[0] == -1                  # negative radiance
    bad_di = ocr.request(sid, 0, mode="di", light=lt, out=1, albedo=float("nan"))
    assert srv.try_submit(bad_di)[0] == -1                  # non-finite albedo
    lt.pdf = 7
    assert srv.try_submit(ocr.request(sid, 0, mode="shadow_sa", light=lt, out=1))[0] == -1  # unknown density
    with pytest.raises(ocr.OcrError):
        ocr.Server(100, slots=1, mock=True)                  # budget below the minimum
    with pytest.raises(ocr.OcrError):
        ocr.Server(1 << 20, slots=0, mock=True)
    srv.destroy()


def test_server_held_outputs_and_release():
    w, h = 32, 32
    state = 2 * ((12 * w * h + 255) // 256 * 256) + (4 * w * h + 255) // 256 * 256
    outb = (4 * w * h + 255) // 256 * 256
    srv = _server(state + 2 * outb, slots=2, ns_per_px=100.0)  # one at a time; two held outputs fit
    sid = srv.add_scene(None, _views([(w, h)]))
    t1 = srv.submit(_req(sid, 0, out=None))
    t2 = srv.submit(_req(sid, 0, out=None))
    res = _wait_done(srv, 2)
    assert {r.ticket for r in res} == {t1, t2}
    assert res[0].out != res[1].out  # distinct arena slices
    # both outputs held: a third request cannot start until one is released
    t3 = srv.submit(_req(sid, 0, out=None))
    time.sleep(0.05)
    assert srv.stats().queued == 1
    with pytest.raises(ocr.OcrError):
        srv.drain()  # would wait forever on the held outputs
    srv.release(t1)
    r3 = _wait_done(srv, 1)
    assert r3[0].ticket == t3
    with pytest.raises(ocr.OcrError):
        srv.release(t1)  # already given back
    srv.release(t2)
    srv.release(t3)
    srv.destroy()


def test_latency_statistics():
    srv = _server(1 << 30, slots=2, ns_per_px=1000.0)  # 32x32 -> ~1 ms
    sid = srv.add_scene(None, _views([(32, 32)]))
    now = ocr.server_now_ms()
    for i in range(20):
        srv.submit(_req(sid, 0, seed=i, arrival_ms=now))
    res = _wait_done(srv, 20)
    st = srv.stats()
    lat = sorted(r.latency_ms for r in res)
    assert all(abs(r.latency_ms - (r.end_ms - r.arrival_ms)) < 1e-9 for r in res)
    assert lat[0] >= 1.0 - 1e-6  # at least the service time
    assert st.p50_ms == pytest.approx(lat[9])   # nearest rank: ceil(0.5 * 20) = 10th
    assert st.p99_ms == pytest.approx(lat[19])
    assert st.max_ms == pytest.approx(lat[-1])
    assert st.frames_per_s > 0
    srv.destroy()


def test_destroy_with_queued_work():
    srv = _server(1 << 30, slots=1, ns_per_px=100.0)
    sid = srv.add_scene(None, _views([(32, 32)]))
    for i in range(10):
        srv.submit(_req(sid, 0, seed=i))
    srv.destroy()  # drains before returning


def test_injected_faults_release_memory_and_server_carries_on():
    w, h = 32, 32
    state = 2 * ((12 * w * h + 255) // 256 * 256) + (4 * w * h + 255) // 256 * 256
    outb = (4 * w * h + 255) // 256 * 256
    # room for one request and one held output: a failed request that kept
    # its state or output would leave every later one waiting for ever
    srv = _server(state + outb, slots=2, ns_per_px=200.0, fault_every=3)
    sid = srv.add_scene(None, _views([(w, h)]))
    results = []
    for i in range(9):
        t = srv.submit(_req(sid, 0, seed=i, out=None))
        r = _wait_done(srv, 1)[0]
        assert r.ticket == t
        results.append(r)
        if r.status == 0:
            srv.release(t)  # make room for the next
        else:
            with pytest.raises(ocr.OcrError):
                srv.release(t)  # a failed request holds no output
    assert [r.status for r in results] == [0, 0, -2] * 3  # OCR_ERR_OOM on every third admission
    st = srv.stats()
    assert st.completed == 9 and st.failed == 3 and st.queued == 0 and st.in_flight == 0
    assert st.peak_bytes <= st.budget_bytes
    # latency statistics cover the successful requests only
    ok = sorted(r.latency_ms for r in results if r.status == 0)
    assert st.max_ms == pytest.approx(ok[-1])
    # a burst with faults: every request completes, the failures in admission order
    for i in range(12):
        srv.submit(_req(sid, 0, seed=i))
    res = sorted(_wait_done(srv, 12), key=lambda r: r.ticket)
    assert [r.status for r in res] == [0, 0, -2] * 4
    assert srv.stats().failed == 7
    srv.destroy()


def test_fault_every_must_not_be_negative():
    with pytest.raises(ocr.OcrError):
        _server(1 << 20, slots=1, fault_every=-1)
