"""Parity of the HIP finder (through the C ABI) with the CPU oracle.

Every comparison is exact: the candidates' integer fields, their float bin
centres and the ordered hit lists must be identical, as must the debug
histograms. Inputs come from the seeded generator only.
"""
import numpy as np
import pytest

from oracle import OracleConfig, oracle_acc_after, oracle_find, oracle_find_batch, oracle_tables
from paper_2511_02742_amd import eventgen

pytestmark = pytest.mark.gpu

FIELDS = ["event", "iter", "theta_bin", "rho_bin", "peak_votes", "n_hits", "hit_offset", "theta", "rho"]


def _ocfg(hcfg) -> OracleConfig:
    return OracleConfig(n_theta=hcfg.n_theta, n_rho=hcfg.n_rho, rho_min=hcfg.rho_min, rho_max=hcfg.rho_max,
                        n_vanes=hcfg.n_vanes, phi_unit=hcfg.phi_unit, min_votes=hcfg.min_votes,
                        peak_mode=hcfg.peak_mode, nms_radius=hcfg.nms_radius,
                        assoc_window=hcfg.assoc_window, max_iters=hcfg.max_iters,
                        coarse_theta=hcfg.coarse_theta or 10, coarse_rho=hcfg.coarse_rho or 10)


_finders = {}


def finder(**kw):
    from paper_2511_02742_amd.hough import HoughFinder
    key = tuple(sorted(kw.items()))
    if key not in _finders:
        _finders[key] = HoughFinder(0, **kw)
    return _finders[key]


def assert_same(gpu, orc, what=""):
    cand, hits, info = gpu
    assert info["status"] == 0, (what, info)
    assert info["candidates"] == len(orc.cand), (what, info["candidates"], len(orc.cand))
    assert info["hits"] == len(orc.hit_index), what
    for f in FIELDS:
        assert np.array_equal(cand[f], orc.cand[f]), (what, f, cand[f][:8], orc.cand[f][:8])
    assert np.array_equal(hits, orc.hit_index), what


def run_batch(f, batch):
    return f.find_host(batch.z, batch.vane, batch.offsets)


def check_batch(batch, what="", **kw):
    f = finder(**kw)
    got = run_batch(f, batch)
    want = oracle_find_batch(_ocfg(f.config), batch.offsets, batch.z, batch.vane)
    assert_same(got, want, what)
    return got, want


def test_tables_byte_equal(gpu_available):
    for kw in ({}, {"n_theta": 512, "n_rho": 512}, {"n_theta": 180, "n_rho": 1000, "phi_unit": 1}):
        f = finder(**kw)
        mine = f.tables()
        ref = oracle_tables(_ocfg(f.config))
        for a, b in zip(mine, ref):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_tiny_event_512(gpu_available):
    e = eventgen.tiny_event(0)
    b = eventgen.make_batch([e])
    got, want = check_batch(b, "tiny", n_theta=512, n_rho=512)
    assert len(want.cand) >= 1


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_pileup50_single_event(gpu_available, seed):
    b = eventgen.make_batch([eventgen.pileup_event(seed)])
    check_batch(b, "pileup50 seed %d" % seed)


@pytest.mark.parametrize("iters", [0, 1, 2, 3])
def test_debug_accumulator(gpu_available, iters):
    for kw, e in (({}, eventgen.pileup_event(7)), ({"n_theta": 512, "n_rho": 512}, eventgen.tiny_event(4)),
                  ({"peak_mode": 0}, eventgen.pileup_event(8))):
        f = finder(**kw)
        acc, info = f.debug_accumulator(e.z, e.vane, iters)
        assert info["status"] == 0
        want = oracle_acc_after(_ocfg(f.config), e.z, e.vane, iters)
        assert np.array_equal(acc, want), (kw, iters)


def test_argmax_mode(gpu_available):
    b = eventgen.pileup_batch(6, seed0=40)
    got, want = check_batch(b, "argmax", peak_mode=0)
    assert np.array_equal(got[0]["n_hits"], got[0]["peak_votes"])


@pytest.mark.parametrize("pileup", [1, 10, 25, 50, 100, 150])
def test_pileup_levels(gpu_available, pileup):
    b = eventgen.pileup_batch(12, n_tracks=pileup, seed0=1000 * pileup)
    check_batch(b, "pileup %d" % pileup)


@pytest.mark.parametrize("assoc_window", [0, 1])
def test_every_register_batch_width(gpu_available, assoc_window):
    # hit counts on both sides of every 64-hit chunk boundary up to one
    # register batch (512 hits): each chunk count of the masks and the
    # recount and each word count of the one-wave claims is taken, batched
    # and as single-event calls
    sizes = [6, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256, 257, 319, 320, 321,
             383, 384, 385, 447, 448, 449, 511, 512]
    evs = []
    for i, n in enumerate(sizes):
        e = eventgen.pileup_event(9000 + i, n_tracks=120)
        assert e.n_hits >= n
        e.z, e.vane, e.r, e.track = e.z[:n], e.vane[:n], e.r[:n], e.track[:n]
        evs.append(e)
    got, want = check_batch(eventgen.make_batch(evs), "widths", assoc_window=assoc_window)
    assert len(want.cand) > len(sizes)
    for n, e in zip(sizes, evs):
        check_batch(eventgen.make_batch([e]), "width %d alone" % n, assoc_window=assoc_window)


def order_edge_events(n_events, seed0=9500):
    """Events that stress the longest-first ordering: empty, one-hit, above
    1023 hits (one shared bucket of the ordering sort) and many of one size."""
    evs = []
    for i in range(n_events):
        kind = i % 7
        if kind == 0:
            e = eventgen.make_event(1, 0, noise_frac=0.0)                        # empty
        elif kind == 1:
            e = eventgen.pileup_event(9500 + i)
            e.z, e.vane, e.r, e.track = e.z[:1], e.vane[:1], e.r[:1], e.track[:1]  # one hit
        elif kind == 2:
            e = eventgen.pileup_event(9500 + i, n_tracks=260)                     # above 1023 hits
        else:
            e = eventgen.pileup_event(seed0 + i, n_tracks=50)
            e.z, e.vane, e.r, e.track = e.z[:200], e.vane[:200], e.r[:200], e.track[:200]  # one size
        evs.append(e)
    assert max(e.n_hits for e in evs) > 1023
    return evs


def test_longest_first_order_edge_sizes(gpu_available):
    # a call of more events than resident finder workgroups runs them longest
    # first; every event must come out once, in event order. (630 events: more
    # than the 256 finder workgroups of 1024 threads an MI355X holds at once;
    # the ordered flag fails the test if that stops being so)
    evs = order_edge_events(630)
    got, want = check_batch(eventgen.make_batch(evs), "order edges")
    assert len(want.cand) > 0
    assert got[2]["ordered"] == 1, got[2]
    # a call of no more events than resident workgroups is not ordered
    got, _ = check_batch(eventgen.make_batch(evs[:200]), "order edges, 200 events")
    assert got[2]["ordered"] == 0, got[2]


def test_uneven_batch(gpu_available):
    b = eventgen.poisson_batch(256)
    check_batch(b, "poisson batch")


def test_batched_equals_alone(gpu_available):
    b = eventgen.poisson_batch(48, seed0=5000)
    f = finder()
    cand, hits, info = run_batch(f, b)
    for e_id in range(b.n_events):
        one = eventgen.make_batch([b.events[e_id]])
        c1, h1, i1 = run_batch(f, one)
        sel = cand["event"] == e_id
        ce = cand[sel]
        assert len(ce) == len(c1)
        for fld in FIELDS:
            if fld in ("event", "hit_offset"):
                continue
            assert np.array_equal(ce[fld], c1[fld])
        if len(ce):
            base = ce["hit_offset"][0]
            assert np.array_equal(ce["hit_offset"] - base, c1["hit_offset"])
            assert np.array_equal(hits[base:base + len(h1)], h1)


@pytest.mark.parametrize("kw", [{"wg_threads": 256}, {"wg_threads": 512}, {"tile_rows": 8},
                                {"tile_rows": 17, "wg_threads": 512}, {"nms_radius": 0},
                                {"nms_radius": 2}, {"assoc_window": 1}, {"phi_unit": 1},
                                {"n_theta": 180, "n_rho": 1000}, {"max_iters": 1},
                                {"sweep_groups": 1}, {"sweep_groups": 16}, {"sweep_groups": 3, "sweep_threads": 1024},
                                {"sweep_groups": 8, "peak_mode": 0}, {"sweep_groups": 4, "wg_threads": 512}])
def test_config_variants(gpu_available, kw):
    b = eventgen.pileup_batch(8, seed0=300)
    check_batch(b, str(kw), **kw)


def test_edge_events(gpu_available):
    evs = []
    evs.append(eventgen.make_event(1, 5, noise_frac=0.0))            # 0 hits with this seed
    base = eventgen.pileup_event(9)
    e1 = eventgen.make_event(1, 0, noise_frac=0.0)
    evs.append(e1)                                                    # no tracks at all
    one = eventgen.pileup_event(10)
    one.z, one.vane, one.r, one.track = one.z[:1], one.vane[:1], one.r[:1], one.track[:1]
    evs.append(one)                                                   # a single hit
    same = eventgen.pileup_event(11)
    same.vane = np.full_like(same.vane, 13)                           # every hit on one vane
    evs.append(same)
    ident = eventgen.pileup_event(12)
    ident.z = np.full_like(ident.z, np.float32(12.35))
    ident.vane = np.full_like(ident.vane, 21)                         # identical hits
    evs.append(ident)
    edge = eventgen.pileup_event(13)
    edge.z = np.zeros_like(edge.z)
    edge.vane = np.zeros_like(edge.vane)                              # rho = 0 on a bin edge
    evs.append(edge)
    evs.append(base)
    big = eventgen.pileup_event(14, n_tracks=100)                    # more hits than one register batch
    evs.append(big)
    b = eventgen.make_batch(evs)
    assert big.n_hits > 512
    check_batch(b, "edges")
    check_batch(b, "edges 1000 bins", n_theta=180, n_rho=1000)
    check_batch(b, "edges argmax", peak_mode=0)
    check_batch(b, "edges split sweep", sweep_groups=8)
    for e in evs:
        check_batch(eventgen.make_batch([e]), "edge alone", sweep_groups=8)


def test_overflowing_hot_and_peak_lists(gpu_available):
    # T = 2 with thousands of hits: every tile overflows the hot list and the
    # peak list is truncated, so the histogram is swept several times.
    rng = np.random.default_rng(9)
    n = 3000
    z = rng.uniform(-200, 200, n).astype(np.float32)
    v = rng.integers(0, 40, n).astype(np.int16)
    e = eventgen.pileup_event(1)
    e.z, e.vane = z, v
    e.r = np.zeros(n, np.float32)
    e.track = np.zeros(n, np.int32)
    b = eventgen.make_batch([e])
    got, want = check_batch(b, "overflow", n_theta=64, n_rho=256, min_votes=2)
    info = got[2]
    # the tiled fallback ran, its peak list was truncated and re-swept, and
    # hot lists overflowed into full tile scans
    assert info["tiled"] > 0 and info["truncations"] > 0 and info["hot_scans"] > 0, info
    assert info["passes"] > info["iters"] - info["recounts"], info
    check_batch(b, "overflow argmax", n_theta=64, n_rho=256, min_votes=3, peak_mode=0, max_iters=20)
    check_batch(b, "overflow T=1", n_theta=32, n_rho=128, min_votes=1, max_iters=3)


def test_hot_set_overflow_takes_the_large_path(gpu_available):
    # few enough hits for the row-stream sweep, but far more bins reach T than
    # the LDS hot set holds: the iteration is redone with the hot set, the
    # window test and the peak list in a device-memory slot. A lone event of
    # more than 448 hits has its first band swept ahead by k_band instead, so
    # its first iteration takes the large-event path at once
    rng = np.random.default_rng(10)
    for n, overflow in ((440, True), (480, False)):
        e = eventgen.pileup_event(2)
        e.z = rng.uniform(-200, 200, n).astype(np.float32)
        e.vane = rng.integers(0, 40, n).astype(np.int16)
        e.r = np.zeros(n, np.float32)
        e.track = np.zeros(n, np.int32)
        b = eventgen.make_batch([e])
        got, want = check_batch(b, "hot set overflow %d" % n, n_theta=64, n_rho=256, min_votes=2)
        assert (got[2]["hotset_full"] > 0) == overflow and got[2]["large"] > 0 and got[2]["tiled"] == 0, got[2]


def test_unsafe_hits_take_the_tiled_path(gpu_available):
    # a rho range narrower than the hits reach: some votes fall outside the
    # histogram, so the streamed paths (which assume every vote lands) are
    # not used and the tiled sweep with its range test runs
    b = eventgen.pileup_batch(6, seed0=1700)
    b2 = eventgen.make_batch([eventgen.pileup_event(1710, n_tracks=100)])
    for batch in (b, b2):
        got, want = check_batch(batch, "narrow rho", rho_min=-300.0, rho_max=300.0)
        assert got[2]["tiled"] > 0 and got[2]["large"] == 0, got[2]


@pytest.mark.parametrize("pileup,n_events", [(100, 8), (150, 4)])
def test_large_events(gpu_available, pileup, n_events):
    # more alive hits than the registers hold and more bins >= T and peaks
    # than LDS holds: the large-event path (hits beyond 512 in LDS, hot set,
    # hash table and peak list in a device-memory slot)
    b = eventgen.pileup_batch(n_events, n_tracks=pileup, seed0=7000 + pileup)
    assert max(np.diff(b.offsets)) > 512
    got, want = check_batch(b, "pileup %d" % pileup)
    assert got[2]["large"] > 0 and got[2]["tiled"] == 0, got[2]
    for e in range(min(2, n_events)):
        one = eventgen.make_batch([b.events[e]])
        got1, _ = check_batch(one, "pileup %d alone" % pileup)
        assert got1[2]["tiled"] == 0, got1[2]


@pytest.mark.parametrize("kw", [{}, {"wg_threads": 512, "tile_rows": 14}, {"wg_threads": 256, "tile_rows": 6}])
def test_small_call_large_events_mixed(gpu_available, kw):
    # a call of a few events takes its large events' first banded sweep
    # ahead of the finder, one workgroup per finder wave, each large event in
    # its own reserved slot; small events, large events of different sizes
    # and the last event large, in one call
    evs = [eventgen.pileup_event(7600, n_tracks=100), eventgen.pileup_event(7601, n_tracks=10),
           eventgen.pileup_event(7602, n_tracks=150), eventgen.pileup_event(7603, n_tracks=50),
           eventgen.pileup_event(7604, n_tracks=120)]
    b = eventgen.make_batch(evs)
    assert sum(int(n) > 512 for n in np.diff(b.offsets)) == 3
    got, want = check_batch(b, "small mixed call " + str(kw), **kw)
    assert got[2]["large"] > 0, got[2]
    if not kw:
        assert got[2]["tiled"] == 0, got[2]
    # the same call twice on one finder: the reserved slots are released
    f = finder(**kw)
    first = run_batch(f, b)
    again = run_batch(f, b)
    assert_same(again, want, "small mixed call again " + str(kw))
    assert_same(first, want, "small mixed call first " + str(kw))


@pytest.mark.parametrize("kw", [{}, {"wg_threads": 512, "tile_rows": 14}])
def test_small_call_band_below_register_batch(gpu_available, kw):
    # events of 449..512 hits (within the register batch, but with more
    # window-test peaks than the finder's LDS list holds): in a call of a few
    # events their first banded sweep is also done ahead by k_band and the
    # finder's first iteration takes the large-event path directly
    evs = [eventgen.pileup_event(7711, n_tracks=90), eventgen.pileup_event(7738, n_tracks=90),
           eventgen.pileup_event(7708, n_tracks=90), eventgen.pileup_event(7601, n_tracks=10),
           eventgen.pileup_event(7604, n_tracks=120)]
    sizes = [int(n) for n in np.diff(eventgen.make_batch(evs).offsets)]
    assert all(448 < n <= 512 for n in sizes[:3]) and sizes[3] < 448 and sizes[4] > 512, sizes
    for e in range(3):
        one = eventgen.make_batch([evs[e]])
        got1, _ = check_batch(one, "band below 512 alone %d %s" % (e, kw), **kw)
        assert got1[2]["large"] > 0 and got1[2]["tiled"] == 0, got1[2]
    got, want = check_batch(eventgen.make_batch(evs), "band below 512 mixed " + str(kw), **kw)
    assert got[2]["large"] >= 4 and got[2]["tiled"] == 0, got[2]


@pytest.mark.parametrize("kw", [{"min_votes": 10}, {"min_votes": 12}, {"min_votes": 12, "wg_threads": 512, "tile_rows": 14}])
def test_large_event_compacted_passes(gpu_available, kw):
    # a large event's first peaks claim most of its hits; its later
    # association passes run over the compacted unclaimed hits. At T = 6 a
    # pileup-150 event leaves a few dozen unclaimed (one 64-hit word); higher
    # thresholds leave a hundred or more (two or three words), which takes
    # the wave-per-peak masks and the multi-word claims of a compacted pass
    b = eventgen.pileup_batch(3, n_tracks=150, seed0=7900)
    got, want = check_batch(b, "compacted passes " + str(kw), **kw)
    assert got[2]["large"] > 0 and got[2]["tiled"] == 0, got[2]
    one = eventgen.make_batch([b.events[0]])
    got1, _ = check_batch(one, "compacted passes alone " + str(kw), **kw)
    assert got1[2]["large"] > 0, got1[2]


@pytest.mark.parametrize("kw", [{"sweep_groups": 4}, {"wg_threads": 512}, {"peak_mode": 0, "max_iters": 12},
                                {"nms_radius": 2}, {"assoc_window": 1}, {"wg_threads": 512, "tile_rows": 14},
                                {"wg_threads": 256, "tile_rows": 6}])
def test_large_event_variants(gpu_available, kw):
    b = eventgen.pileup_batch(3, n_tracks=150, seed0=7300)
    got, want = check_batch(b, "pileup 150 " + str(kw), **kw)
    assert got[2]["large"] > 0, got[2]


def test_recount_iterations_used(gpu_available):
    # pileup events: after the first sweep, later iterations recount the hot
    # set instead of sweeping the histogram again
    b = eventgen.pileup_batch(16, seed0=800)
    got, want = check_batch(b, "recount nms")
    assert got[2]["recounts"] > 0 and got[2]["tiled"] == 0, got[2]
    got, want = check_batch(b, "recount argmax", peak_mode=0)
    assert got[2]["recounts"] >= got[2]["iters"] - 16, got[2]


_full_ref = {}


def full_size_reference(ocfg, b):
    """The oracle's output for every event of a batch (independent processes
    over event slices, concatenated: the same arrays as one batch call)."""
    import os
    from oracle.oracle import oracle_find_batch_sliced
    key = (repr(ocfg), len(b.offsets), int(b.offsets[-1]))
    if key not in _full_ref:
        _full_ref[key] = oracle_find_batch_sliced(ocfg, b.offsets, b.z, b.vane,
                                                  workers=min(16, os.cpu_count() or 1))
    return _full_ref[key]


@pytest.mark.parametrize("kw", [{}, {"sweep_groups": 2}, {"wg_threads": 512, "tile_rows": 14}])
def test_full_size_batch(gpu_available, kw):
    # 4096 pileup-50 events in one launch (the benchmark configuration, run
    # longest event first): every event byte-equal to the oracle
    # ({wg_threads 512, tile_rows 14}: two events' workgroups per CU)
    b = eventgen.pileup_batch(4096)
    f = finder(**kw)
    got = run_batch(f, b)
    assert_same(got, full_size_reference(_ocfg(f.config), b), "full-size batch %s" % kw)


def test_empty_batch(gpu_available):
    b = eventgen.make_batch([])
    f = finder()
    cand, hits, info = run_batch(f, b)
    assert info["status"] == 0 and info["candidates"] == 0 and info["hits"] == 0


@pytest.mark.parametrize("kw", [{}, {"sweep_groups": 4}])
def test_invalid_hits_reported(gpu_available, kw):
    b = eventgen.pileup_batch(4, seed0=60)
    f = finder(**kw)
    vane = b.vane.copy()
    vane[b.offsets[2] + 5] = 40
    cand, hits, info = f.find_host(b.z, vane, b.offsets)
    assert info["status"] == -6 and info["detail"] == b.offsets[2] + 5 and info["candidates"] == 0
    z = b.z.copy()
    z[7] = np.nan
    cand, hits, info = f.find_host(z, b.vane, b.offsets)
    assert info["status"] == -6 and info["detail"] == 7
    # one event alone (single-kernel path)
    one = eventgen.make_batch([b.events[1]])
    vone = one.vane.copy()
    vone[3] = -1
    cand, hits, info = f.find_host(one.z, vone, one.offsets)
    assert info["status"] == -6 and info["detail"] == 3 and info["candidates"] == 0
    # the context keeps working afterwards
    check_batch(b, "after error", **kw)
    check_batch(one, "after error, one event", **kw)


def test_capacity_checked_on_host(gpu_available):
    import torch
    from paper_2511_02742_amd.hough import HOUGH_ERR_CAPACITY, HoughError
    b = eventgen.pileup_batch(2, seed0=70)
    f = finder()
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    with pytest.raises(HoughError) as ei:
        f.find(z, v, o, capacities=(1, 1))
    assert ei.value.status == HOUGH_ERR_CAPACITY


def test_deterministic_repeats(gpu_available):
    b = eventgen.poisson_batch(128, seed0=900)
    f = finder()
    r0 = run_batch(f, b)
    for _ in range(3):
        r = run_batch(f, b)
        assert np.array_equal(r[0], r0[0]) and np.array_equal(r[1], r0[1])


def _permute_within_events(batch, seed):
    rng = np.random.default_rng(seed)
    z = batch.z.copy()
    v = batch.vane.copy()
    for e in range(batch.n_events):
        lo, hi = batch.offsets[e], batch.offsets[e + 1]
        p = lo + rng.permutation(hi - lo)
        z[lo:hi] = batch.z[p]
        v[lo:hi] = batch.vane[p]
    return z, v


@pytest.mark.parametrize("kw,n_events", [({}, 96), ({"sweep_groups": 2}, 96), ({}, 1)])
def test_graph_replays_match_oracle(gpu_available, kw, n_events):
    # captured launch: replays with eager work and synchronisations between
    # them, the input buffers rewritten between replays; every replay is
    # checked against the oracle of the data it saw
    import torch
    b = eventgen.poisson_batch(n_events, seed0=7000)
    f = finder(**kw)
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    g = f.capture(z, v, o)
    other = eventgen.pileup_batch(3, seed0=7100)
    ocfg = _ocfg(f.config)
    for rep in range(4):
        zz, vv = (b.z, b.vane) if rep == 0 else _permute_within_events(b, rep)
        z.copy_(torch.from_numpy(zz))
        v.copy_(torch.from_numpy(vv))
        out = g.launch()
        torch.cuda.synchronize(dev)
        got = out.to_host()
        want = oracle_find_batch(ocfg, b.offsets, zz, vv)
        assert_same(got, want, "replay %d" % rep)
        # eager work on the same context between replays
        check_batch(other, "eager between replays", **kw)
    g.close()


@pytest.mark.parametrize("kw", [{}, {"n_theta": 180, "n_rho": 1000, "peak_mode": 2}])
def test_graph_replays_ordered_call(gpu_available, kw):
    # a captured call of more events than resident finder workgroups (so the
    # ordering kernel is captured too), mixed sizes; every replay against the
    # oracle, eager calls on the same context between replays
    import torch
    f = finder(**kw)
    n_ev = 630 if kw.get("peak_mode", 1) != 2 else 2600
    b = eventgen.make_batch(order_edge_events(n_ev, seed0=12000))
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    want = oracle_find_batch(_ocfg(f.config), b.offsets, b.z, b.vane)
    other = eventgen.pileup_batch(3, seed0=12100)
    g = f.capture(z, v, o)
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize(dev)
        got = out.to_host()
        assert_same(got, want, "ordered replay %d" % rep)
        assert got[2]["ordered"] == 1, got[2]
        check_batch(other, "eager between replays", **kw)
    g.close()


def test_graph_replays_small_call_large_events(gpu_available):
    # a captured call of a few events, three of them large: the large events'
    # first banded sweep (k_band, with its reserved slots) is in the graph;
    # every replay against the oracle, with the hits rewritten between replays
    # and eager calls of large events on the same context in between
    import torch
    f = finder()
    evs = [eventgen.pileup_event(7700 + i, n_tracks=nt) for i, nt in enumerate((100, 25, 150, 50, 110))]
    b = eventgen.make_batch(evs)
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    g = f.capture(z, v, o)
    other = eventgen.make_batch([eventgen.pileup_event(7750, n_tracks=100), eventgen.pileup_event(7751)])
    ocfg = _ocfg(f.config)
    for rep in range(4):
        zz, vv = (b.z, b.vane) if rep == 0 else _permute_within_events(b, rep)
        z.copy_(torch.from_numpy(zz))
        v.copy_(torch.from_numpy(vv))
        out = g.launch()
        torch.cuda.synchronize(dev)
        got = out.to_host()
        want = oracle_find_batch(ocfg, b.offsets, zz, vv)
        assert_same(got, want, "small-call replay %d" % rep)
        assert got[2]["large"] > 0, got[2]
        check_batch(other, "eager large events between replays")
    g.close()


def test_event_clock_stamps(gpu_available):
    # per-event device clock stamps: set for calls up to 128 events, every
    # event stamped with start <= retire inside the call's span; outputs
    # unchanged; a larger call writes none; turned off, nothing is written
    import torch
    from paper_2511_02742_amd.hough import clock_rate
    f = finder()
    dev = torch.device("cuda", 0)
    rate = clock_rate(0)
    assert 1e6 <= rate <= 1e10
    b = eventgen.poisson_batch(96, seed0=12500)
    stamps = torch.zeros(2 * 128, dtype=torch.int64, device=dev)
    f.set_event_clock(stamps)
    try:
        check_batch(b, "with clock stamps")
        s = stamps.cpu().numpy().reshape(-1, 2)
        assert np.all(s[:96, 0] > 0) and np.all(s[:96, 1] >= s[:96, 0]), s[:4]
        assert np.all(s[96:] == 0)
        span = (s[:96, 1].max() - s[:96, 0].min()) / rate
        assert 0 < span < 1.0, span
        # one-event calls stamp event 0
        stamps.zero_()
        check_batch(eventgen.make_batch([b.events[3]]), "one event with clock stamps")
        s = stamps.cpu().numpy().reshape(-1, 2)
        assert s[0, 0] > 0 and s[0, 1] >= s[0, 0] and np.all(s[1:] == 0)
        # a call of more events than the buffer holds writes nothing
        stamps.zero_()
        check_batch(eventgen.poisson_batch(200, seed0=12600), "above the stamp capacity")
        assert int(stamps.abs().sum()) == 0
    finally:
        f.set_event_clock(None)
    check_batch(b, "stamps off")
    assert int(stamps.abs().sum()) == 0


def test_autotune_picks_a_shape_that_matches(gpu_available):
    import torch
    from paper_2511_02742_amd.hough import HoughFinder, autotune
    b = eventgen.poisson_batch(128, seed0=7200)
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    best, ms, tried = autotune(z, v, o, repeats=1)
    assert tried >= 20 and ms > 0
    f = HoughFinder(0, config=best)
    got = f.find_host(b.z, b.vane, b.offsets)
    assert_same(got, oracle_find_batch(_ocfg(f.config), b.offsets, b.z, b.vane), "autotuned")


def test_lds_peak_probe(gpu_available):
    # the roofline denominator: both patterns run and the conflict-free one
    # is the faster
    from paper_2511_02742_amd.hough import lds_peak
    p0, p1 = lds_peak(0), lds_peak(1)
    assert p0 > 0 and p1 > 0 and p0 >= p1


def test_vote_count_is_the_sweeps(gpu_available):
    # one full sweep per event of the pileup-50 set: every hit votes once per
    # theta row in the first iteration, and later iterations recount
    b = eventgen.pileup_batch(64, seed0=8100)
    f = finder()
    _, _, info = run_batch(f, b)
    assert info["votes"] >= b.n_hits * f.config.n_theta and info["votes"] <= info["evals"]
