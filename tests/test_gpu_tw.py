"""Parity of the time-sliced finder with track extension (hough_tw_find,
through the C ABI) with the oracle: tracks (every field) and their ordered
hit lists byte-equal, and the Hough-candidate and continuation counts, on
timelines at the paper's three decay rates, batches of one and of many
timelines, the oracle pins' exact curves, configuration variants and
invalid input. Inputs come from the seeded generator only."""
import numpy as np
import pytest

from oracle import OracleConfig, TwConfig, oracle_tw_find_batch
from paper_2511_02742_amd import eventgen
from test_gpu_parity import _ocfg, finder

pytestmark = pytest.mark.gpu


def _tw(**kw):
    from paper_2511_02742_amd.hough import tw_config
    return tw_config(**kw)


def _otw(tw):
    return TwConfig(window_ns=tw.window_ns, step_ns=tw.step_ns, gate_r=tw.gate_r_mm, gate_z=tw.gate_z_mm,
                    gate_t=tw.gate_t_ns, max_track_hits=tw.max_track_hits)


def check(batch, what="", n_windows=None, tw_kw=None, **kw):
    f = finder(**kw)
    tw = _tw(**(tw_kw or {}))
    if n_windows is None:
        n_windows = batch.n_windows(tw.window_ns, tw.step_ns)
    tracks, hits, info = f.tw_find_host(batch, n_windows=n_windows, tw=tw)
    want = oracle_tw_find_batch(_ocfg(f.config), _otw(tw), batch.offsets, batch.r, batch.z, batch.vane, batch.t,
                                n_windows)
    assert info["status"] == 0, (what, info)
    assert info["tracks"] == len(want.tracks) and info["hits"] == len(want.hit_index), (what, info,
                                                                                      len(want.tracks))
    for fld in want.tracks.dtype.names:
        assert np.array_equal(tracks[fld], want.tracks[fld]), (what, fld)
    assert np.array_equal(hits, want.hit_index), what
    assert info["candidates"] == want.n_candidates and info["continued"] == want.n_carried, (what, info)
    assert info["windows"] == n_windows
    return tracks, hits, info


@pytest.mark.parametrize("rate,span,n_tl", [(6.0, 80.0, 4), (0.6, 500.0, 3), (0.06, 3000.0, 2)])
def test_timelines_at_the_paper_rates(gpu_available, rate, span, n_tl):
    b = eventgen.timeline_batch(n_tl, rate, span, seed0=int(rate * 1000) + 31)
    tracks, _, info = check(b, "rate %g" % rate)
    assert len(tracks) > 0


def test_one_timeline(gpu_available):
    # one window event per step: the finder's single-event path
    b = eventgen.timeline_batch(1, 6.0, 60.0, seed0=77)
    tracks, _, info = check(b, "one timeline")
    assert info["continued"] > 0


def test_many_timelines(gpu_available):
    # 300 timelines: more window events than resident finder workgroups, so
    # the finder orders them longest first
    b = eventgen.timeline_batch(300, 6.0, 22.0, seed0=900)
    check(b, "300 timelines")


def test_exact_curves_of_the_oracle_pins(gpu_available):
    from test_tw_oracle import curve
    tls = []
    for (n, dt, t0, v0) in ((10, 0.2, 1.0, 5), (12, 1.0, 2.0, 7), (10, 0.2, 1.0, 36), (12, 0.25, 6.0, 20)):
        r, z, v, t = curve(n, v0=v0, dt=dt, t0=t0)
        tl = eventgen.Timeline(r=r.astype(np.float32), z=z.astype(np.float32), vane=v.astype(np.int16),
                               t=t.astype(np.float32), track=np.zeros(n, np.int32), seed=0, rate_per_ns=0.0,
                               span_ns=0.0, t_decay=np.zeros(1), p=np.zeros(1))
        tls.append(tl)
    b = eventgen.make_timeline_batch(tls)
    tracks, hits, info = check(b, "pin curves")
    assert list(tracks["n_hits"]) == [10, 12, 10, 12] and list(tracks["carried"]) == [0, 1, 0, 0]


@pytest.mark.parametrize("tw_kw", [{"gate_t_ns": 6.0}, {"max_track_hits": 5}, {"gate_r_mm": 2.0, "gate_z_mm": 1.0},
                                   {"window_ns": 20.0, "step_ns": 10.0}])
def test_configuration_variants(gpu_available, tw_kw):
    b = eventgen.timeline_batch(3, 6.0, 60.0, seed0=1200)
    tracks, _, _ = check(b, "tw %s" % tw_kw, tw_kw=tw_kw)
    if "max_track_hits" in tw_kw:
        assert tracks["n_hits"].max() <= 5


@pytest.mark.parametrize("kw", [{"peak_mode": 0}, {"n_theta": 512, "n_rho": 512}, {"min_votes": 4}])
def test_hough_configuration_variants(gpu_available, kw):
    b = eventgen.timeline_batch(2, 6.0, 50.0, seed0=1300)
    check(b, "hough %s" % kw, **kw)


def test_edge_timelines(gpu_available):
    empty = eventgen.make_timeline(5, 0.0, 50.0)
    assert empty.n_hits == 0
    tls = [eventgen.make_timeline(1400, 6.0, 30.0), empty, eventgen.make_timeline(1401, 0.06, 200.0),
           eventgen.make_timeline(1402, 6.0, 30.0)]
    b = eventgen.make_timeline_batch(tls)
    check(b, "with an empty timeline")
    check(b, "no windows", n_windows=0)
    check(b, "fewer windows than the hits span", n_windows=3)
    check(eventgen.make_timeline_batch([]), "no timelines", n_windows=4)


def test_invalid_hits_reported(gpu_available):
    b = eventgen.timeline_batch(3, 6.0, 30.0, seed0=1500)
    f = finder()
    for what, fix in (("unsorted", lambda t: t.__setitem__(b.offsets[1] + 10, t[b.offsets[1] + 9] - 1.0)),
                      ("negative", lambda t: t.__setitem__(b.offsets[2], -1.0)),
                      ("nan", lambda t: t.__setitem__(b.offsets[1] + 3, np.nan))):
        t = b.t.copy()
        fix(t)
        bad = eventgen.TimelineBatch(r=b.r, z=b.z, vane=b.vane, t=t, offsets=b.offsets, timelines=b.timelines)
        tracks, hits, info = f.tw_find_host(bad, n_windows=8)
        assert info["status"] == -6 and info["tracks"] == 0, (what, info)
        first = int(np.nonzero(~(np.isfinite(t) & (t >= 0)) | np.r_[False, np.diff(t) < 0] & ~np.isin(
            np.arange(len(t)), b.offsets))[0][0])
        assert info["detail"] == first, (what, info["detail"], first)
    # the context works normally afterwards
    check(b, "after errors")
