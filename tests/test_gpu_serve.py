"""Served form (hough_server_* through the C ABI): every request's result is
byte-identical to a one-event call on the same hits and to the oracle,
whatever else shares its launch; arrivals, refusals and back-pressure."""
import numpy as np
import pytest

from oracle import OracleConfig, oracle_find
from paper_2511_02742_amd import eventgen

pytestmark = pytest.mark.gpu

FIELDS = ["event", "iter", "theta_bin", "rho_bin", "peak_votes", "n_hits", "hit_offset", "theta", "rho"]


def _ocfg(hcfg) -> OracleConfig:
    return OracleConfig(n_theta=hcfg.n_theta, n_rho=hcfg.n_rho, rho_min=hcfg.rho_min, rho_max=hcfg.rho_max,
                        n_vanes=hcfg.n_vanes, phi_unit=hcfg.phi_unit, min_votes=hcfg.min_votes,
                        peak_mode=hcfg.peak_mode, nms_radius=hcfg.nms_radius,
                        assoc_window=hcfg.assoc_window, max_iters=hcfg.max_iters)


def _event(batch, e):
    b, n = batch.offsets[e], batch.offsets[e + 1]
    return batch.z[b:n], batch.vane[b:n]


def _collect(srv, n, timeout=60.0):
    import time
    got = {}
    t_end = time.time() + timeout
    while len(got) < n and time.time() < t_end:
        for r in srv.poll():
            assert r.tag not in got
            got[r.tag] = r
        if len(got) < n:
            time.sleep(0.001)
    assert len(got) == n, (len(got), n, srv.stats())
    return got


def _same(r, cand, hits, what):
    assert r.status == 0, (what, r.rec)
    assert len(r.cand) == len(cand), (what, len(r.cand), len(cand))
    for f in FIELDS:
        assert np.array_equal(r.cand[f], cand[f]), (what, f)
    assert np.array_equal(r.hit_index, hits), what


@pytest.mark.parametrize("kw", [{"lanes": 3, "max_batch_events": 16},
                                {"lanes": 1, "max_batch_events": 4096},
                                {"lanes": 4, "max_batch_events": 7, "max_batch_hits": 3000}])
def test_served_results_equal_alone_and_oracle(gpu_available, kw):
    from paper_2511_02742_amd.hough import HoughFinder, HoughServer
    batch = eventgen.mixed_pileup_batch(96)
    f = HoughFinder(0)
    ocfg = _ocfg(f.config)
    with HoughServer(0, **kw) as srv:
        tags = np.arange(1000, 1000 + 96, dtype=np.uint64)
        assert srv.submit(batch.z, batch.vane, batch.offsets, tags=tags) == 96
        got = _collect(srv, 96)
        st = srv.stats()
    assert st["completed"] == 96 and st["refused"] == 0
    assert st["launches"] >= (1 if kw["max_batch_events"] >= 96 else 96 // kw["max_batch_events"])
    for e in range(96):
        z, v = _event(batch, e)
        r = got[1000 + e]
        assert r.rec["n_hits"] == len(z)
        cand, hits, info = f.find_host(z, v, np.array([0, len(z)], np.int64))
        _same(r, cand, hits, ("alone", e))
        o = oracle_find(ocfg, z, v)
        _same(r, o.cand, o.hit_index, ("oracle", e))


def test_served_stream_respects_arrival_times(gpu_available):
    from paper_2511_02742_amd.hough import HoughFinder, HoughServer
    batch = eventgen.mixed_pileup_batch(400, seed0=3_000_000)
    n = 400
    rng = np.random.default_rng(7)
    with HoughServer(0, lanes=3) as srv:
        t0 = srv.clock() + 0.02
        arr = t0 + np.cumsum(rng.exponential(1.0 / 20000.0, n))
        assert srv.submit(batch.z, batch.vane, batch.offsets, t_arrival=arr) == n
        got = _collect(srv, n)
        st = srv.stats()
    assert st["completed"] == n
    want = HoughFinder(0).find_host(batch.z, batch.vane, batch.offsets)
    wc, wh, _ = want
    for e in range(n):
        r = got[e]
        assert r.rec["t_admit"] >= r.rec["t_arrival"]
        assert r.rec["t_done"] >= r.rec["t_admit"]
        sel = wc["event"] == e
        c = wc[sel].copy()
        if len(c):
            h0 = c["hit_offset"][0]
            hits = wh[h0:h0 + int(c["n_hits"].sum())]
            c["hit_offset"] -= h0
            c["event"] = 0
        else:
            hits = wh[:0]
        _same(r, c, hits, ("stream", e))


def test_served_refusals_and_mixed_good_requests(gpu_available):
    from paper_2511_02742_amd.hough import HOUGH_ERR_CAPACITY, HOUGH_ERR_DATA, HoughServer
    good = eventgen.pileup_event(5)
    big = eventgen.pileup_event(6, n_tracks=100)
    z = np.concatenate([good.z, good.z, big.z, good.z]).astype(np.float32)
    v = np.concatenate([good.vane, good.vane, big.vane, good.vane]).astype(np.int16)
    n1 = len(good.z)
    v[n1 + 3] = 99                                   # request 1: invalid vane
    z[-1] = np.nan                                   # request 3: non-finite z
    offs = np.array([0, n1, 2 * n1, 2 * n1 + len(big.z), 3 * n1 + len(big.z)], np.int64)
    with HoughServer(0, max_batch_hits=400) as srv:   # request 2 (pileup 100) is too big
        assert len(big.z) > 400
        assert srv.submit(z, v, offs) == 4
        got = _collect(srv, 4)
        st = srv.stats()
    assert got[0].status == 0 and got[0].rec["lane"] >= 0 and len(got[0].cand) > 0
    assert got[1].status == HOUGH_ERR_DATA and got[1].rec["lane"] == -1
    assert got[2].status == HOUGH_ERR_CAPACITY and got[2].rec["lane"] == -1
    assert got[3].status == HOUGH_ERR_DATA
    assert st["refused"] == 3 and st["submitted"] == 1


def test_served_queue_back_pressure(gpu_available):
    from paper_2511_02742_amd.hough import HoughServer
    batch = eventgen.pileup_batch(10, seed0=40)
    with HoughServer(0, queue_events=4) as srv:
        far = np.full(10, srv.clock() + 3600.0)      # not admitted during the test
        assert srv.submit(batch.z, batch.vane, batch.offsets, t_arrival=far) == 4
        st = srv.stats()
        assert st["pending_events"] == 4 and st["launches"] == 0
        assert srv.submit(batch.z, batch.vane, batch.offsets[:2], t_arrival=far[:1]) == 0


def test_served_empty_requests(gpu_available):
    from paper_2511_02742_amd.hough import HoughServer
    z = np.zeros(0, np.float32)
    v = np.zeros(0, np.int16)
    with HoughServer(0) as srv:
        assert srv.submit(z, v, np.zeros(4, np.int64)) == 3
        got = _collect(srv, 3)
    for t in range(3):
        assert got[t].status == 0 and len(got[t].cand) == 0 and len(got[t].hit_index) == 0


def test_served_poll_reports_a_result_too_large(gpu_available):
    import ctypes
    from paper_2511_02742_amd.hough import HOUGH_ERR_CAPACITY, HoughServer, cand_dtype, served_dtype
    ev = eventgen.pileup_event(11)
    with HoughServer(0) as srv:
        assert srv.submit(ev.z, ev.vane, np.array([0, ev.n_hits], np.int64)) == 1
        srv.drain(60.0)
        recs = np.zeros(1, served_dtype)
        cand = np.zeros(1, cand_dtype)
        hits = np.zeros(4, np.int32)
        k = ctypes.c_int32(-1)
        st = srv._lib.hough_server_poll(srv._h, 1, recs.ctypes.data, cand.ctypes.data, 1, hits.ctypes.data, 4,
                                        ctypes.byref(k))
        assert st == HOUGH_ERR_CAPACITY and k.value == 0
        got = _collect(srv, 1)
    assert got[0].status == 0 and len(got[0].cand) > 1


def test_served_admission_by_device_memory(gpu_available):
    # a 2 MiB device arena: a launch's block (its inputs and a workspace for
    # exactly its events and hits, about 0.5 MiB of large-event slot per
    # event here) limits how many requests a launch takes and how many
    # launches run at once; results stay byte-identical to one-event calls,
    # and a request whose launch alone exceeds the arena is refused
    from paper_2511_02742_amd.hough import HOUGH_ERR_CAPACITY, HoughFinder, HoughServer
    batch = eventgen.mixed_pileup_batch(120, levels=(1, 10, 25, 50), seed0=4_100_000)
    arena = 2 << 20
    f = HoughFinder(0)
    with HoughServer(0, lanes=3, device_bytes=arena) as srv:
        assert srv.submit(batch.z, batch.vane, batch.offsets, tags=np.arange(120, dtype=np.uint64)) == 120
        got = _collect(srv, 120)
        st = srv.stats()
        huge = eventgen.make_batch([eventgen.pileup_event(4_200_000 + i, n_tracks=150) for i in range(130)])
        n_big = 100_000
        assert huge.n_hits >= n_big
        assert srv.submit(huge.z[:n_big], huge.vane[:n_big], np.array([0, n_big], np.int64),
                          tags=np.array([999], np.uint64)) == 1
        refused = _collect(srv, 1)[999]
    assert st["device_bytes"] == arena
    assert 0 < st["max_device_bytes_in_use"] <= arena and st["device_bytes_in_use"] == 0
    assert st["launches"] >= 120 // 3 and st["launched_events"] == 120
    assert refused.status == HOUGH_ERR_CAPACITY and refused.rec["lane"] == -1
    for e in range(120):
        z, v = _event(batch, e)
        cand, hits, _ = f.find_host(z, v, np.array([0, len(z)], np.int64))
        _same(got[e], cand, hits, ("arena", e))
