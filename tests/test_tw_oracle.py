"""Pins of the time-sliced track-finding oracle (no GPU): three-point seeds
extended vane by vane inside 10 ns windows sliding by 5 ns, with the
continuation of flagged tracks (paper Sec. 4 and 5). Expected results come
from the definitions: hits on an exact quadratic curve over consecutive
vanes are all found by the extrapolation, gates decide at their
boundaries, windows are half-open, and a track crossing a window edge is
continued instead of being cut."""
import math

import numpy as np
import pytest

from oracle import OracleConfig, TwConfig, oracle_tw_find_batch
from oracle.oracle import OracleError
from paper_2511_02742_amd import eventgen

CFG = OracleConfig()
TW = TwConfig()


def run(r, z, vane, t, n_windows=None, tw=TW):
    r = np.asarray(r, np.float32)
    z = np.asarray(z, np.float32)
    t = np.asarray(t, np.float32)
    vane = np.asarray(vane, np.int16)
    order = np.argsort(t, kind="stable")
    assert np.array_equal(order, np.arange(len(t))), "pins give hits in time order"
    if n_windows is None:
        n_windows = int(math.floor(float(t.max()) / tw.step_ns)) + 1 if len(t) else 0
    return oracle_tw_find_batch(CFG, tw, np.array([0, len(t)], np.int64), r, z, vane, t, n_windows)


def curve(n, v0=5, t0=1.0, dt=0.2, r0=150.0, r1=2.0, r2=0.5, z0=-20.0, z1=3.0):
    """n hits on consecutive vanes v0, v0+1, ... on an exact quadratic r(k)
    and a straight z(k) (so also a straight line in (vane azimuth, z))."""
    k = np.arange(n, dtype=np.float64)
    vane = (v0 + np.arange(n)) % 40
    return (r0 + r1 * k + r2 * k * k), (z0 + z1 * k), vane, (t0 + dt * k)


def hits_of(res, i):
    tr = res.tracks[i]
    return res.hit_index[tr["hit_offset"]:tr["hit_offset"] + tr["n_hits"]]


def test_quadratic_curve_is_found_whole_in_vane_order():
    r, z, v, t = curve(10)
    res = run(r, z, v, t)
    assert len(res.tracks) == 1
    assert np.array_equal(hits_of(res, 0), np.arange(10))
    tr = res.tracks[0]
    assert (tr["vane_first"], tr["vane_last"], tr["window"], tr["carried"]) == (5, 14, 0, 0)


def test_curve_across_vane_zero_and_downward_vanes():
    # vanes 36..39, 0..5: the extension steps over the wrap; hits given in
    # decreasing-vane order of time (the positron's clockwise sense)
    r, z, v, t = curve(10, v0=36)
    res = run(r[::-1].copy(), z[::-1].copy(), v[::-1].copy(), t)
    assert len(res.tracks) == 1
    h = hits_of(res, 0)
    assert np.array_equal(h, np.arange(10)[::-1])       # vane order from the lower end: 36, 37, ...
    assert (res.tracks[0]["vane_first"], res.tracks[0]["vane_last"]) == (36, 5)


@pytest.mark.parametrize("field,off,taken", [("r", 10.0 - 0.25, True), ("r", 10.0 + 0.25, False),
                                             ("z", 4.0 - 0.25, True), ("z", 4.0 + 0.25, False),
                                             ("t", 2.0 - 0.05, True), ("t", 2.0 + 0.05, False)])
def test_gates_decide_at_their_bounds(field, off, taken):
    # 8 hits on the curve, then one hit on the next vane displaced from the
    # extrapolated point by just under or just over a gate
    r, z, v, t = curve(9)
    if field == "r":
        r[8] += off
    elif field == "z":
        z[8] += off
    else:
        t[8] = t[7] + off
    res = run(r, z, v, t)
    assert len(res.tracks) == 1
    assert res.tracks[0]["n_hits"] == (9 if taken else 8)


def test_closest_hit_wins_and_ties_go_to_the_lower_index():
    r, z, v, t = curve(9)
    # two hits on the vane after the curve: one 1.0 mm off in r, one 0.5 mm
    r = np.append(r, r[8] + 0.0)
    z = np.append(z, z[8] + 0.0)
    v = np.append(v, v[8])
    t = np.append(t, t[8])
    r[8] += 1.0
    r[9] += 0.5
    res = run(r, z, v, t)
    assert hits_of(res, 0)[-1] == 9
    # equal distances: the lower index
    r[8] = r[9]
    res = run(r, z, v, t)
    assert hits_of(res, 0)[-1] == 8


def test_seed_takes_the_lowest_index_hit_on_each_vane():
    # a second hit on the first seed vane (vane 5), 0.3 mm off the curve and
    # earlier in hit order than the on-curve one: the seed takes it, the
    # on-curve hit stays out
    r, z, v, t = curve(10)
    r = np.concatenate([[r[0] + 0.3], r])
    z = np.concatenate([[z[0]], z])
    v = np.concatenate([[v[0]], v])
    t = np.concatenate([[t[0] - 0.01], t])
    res = run(r, z, v, t)
    assert len(res.tracks) == 1
    h = hits_of(res, 0)
    assert h[0] == 0 and 1 not in h and len(h) == 10


def test_window_edges_are_half_open():
    # every hit at t = 10.0: windows [5, 15) and [10, 20) hold them, [0, 10) not
    r, z, v, t = curve(10, dt=0.0, t0=10.0)
    res = run(r, z, v, t)
    assert len(res.tracks) == 1 and res.tracks[0]["window"] == 1
    r, z, v, t = curve(10, dt=0.0, t0=np.float32(9.999))
    res = run(r, z, v, t)
    assert res.tracks[0]["window"] == 0


def test_track_across_a_window_edge_is_continued():
    # 12 hits at t = 2, 3, ..., 13 ns: window 0 sees 8 of them (a Hough
    # candidate, a seed, extended to t = 9), window 1 continues the flagged
    # track with the last four; one track of 12 hits, continued once
    r, z, v, t = curve(12, dt=1.0, t0=2.0)
    res = run(r, z, v, t)
    assert len(res.tracks) == 1
    tr = res.tracks[0]
    assert tr["n_hits"] == 12 and tr["window"] == 0 and tr["last_window"] == 1 and tr["carried"] == 1
    assert res.n_carried == 1
    # the same track entirely inside window 1 needs no continuation
    r, z, v, t = curve(12, dt=0.25, t0=6.0)
    res = run(r, z, v, t)
    assert res.tracks[0]["carried"] == 0 and res.tracks[0]["n_hits"] == 12


def test_unflagged_tracks_are_not_continued():
    # the flag needs the track's latest hit at or after the next window's
    # start. With gate_t below window - step that never changes a result
    # (a hit the continuation could take lies in the earlier window too), so
    # a 6 ns time gate: the track ends at t = 4.7 < 5, four later hits on its
    # extrapolation at t = 10.2.. (windows 1 and 2 only, within 6 ns of its
    # end) are not added, and four hits cannot seed a candidate (T = 6)
    tw = TwConfig(gate_t=6.0)
    r, z, v, t = curve(12, dt=0.3, t0=2.6)
    t = t.astype(np.float32)
    t[8:] = np.float32(10.2) + np.float32(0.05) * np.arange(4, dtype=np.float32)
    res = run(r, z, v, t, tw=tw)
    assert len(res.tracks) == 1 and res.tracks[0]["n_hits"] == 8 and res.n_carried == 0
    # ending at t = 5.0 instead, it is flagged and continued to all 12 hits
    t[:8] += np.float32(0.3)
    res = run(r, z, v, t, tw=tw)
    assert len(res.tracks) == 1 and res.tracks[0]["n_hits"] == 12 and res.tracks[0]["carried"] == 1


def test_time_shift_by_whole_steps_shifts_windows_only():
    # (no hits before 5 ns: the shifted run's window 2 would hold them, while
    # the original run has no window before [0, 10))
    tl = eventgen.make_timeline(41, 6.0, 60.0)
    keep = tl.t >= 5.0
    r, z, v = tl.r[keep], tl.z[keep], tl.vane[keep]
    # times on a 1/64 ns grid, so that adding 15 ns is exact in float
    t1 = (np.round(tl.t[keep].astype(np.float64) * 64.0) / 64.0).astype(np.float32)
    n = len(t1)
    a = oracle_tw_find_batch(CFG, TW, np.array([0, n]), r, z, v, t1, 14)
    t2 = (t1.astype(np.float64) + 15.0).astype(np.float32)
    assert np.array_equal(t2 - np.float32(15.0), t1)
    b = oracle_tw_find_batch(CFG, TW, np.array([0, n]), r, z, v, t2, 17)
    assert len(a.tracks) == len(b.tracks) > 0
    assert np.array_equal(a.hit_index, b.hit_index)
    for f in ("n_hits", "vane_first", "vane_last", "theta_bin", "rho_bin", "carried"):
        assert np.array_equal(a.tracks[f], b.tracks[f]), f
    assert np.array_equal(a.tracks["window"] + 3, b.tracks["window"])


def test_invariants_on_generated_timelines():
    for rate, span in ((6.0, 80.0), (0.6, 400.0)):
        b = eventgen.timeline_batch(3, rate, span, seed0=500)
        res = oracle_tw_find_batch(CFG, TW, b.offsets, b.r, b.z, b.vane, b.t, b.n_windows())
        assert len(res.tracks) > 0
        for tl_id in range(3):
            tracks = res.tracks[res.tracks["timeline"] == tl_id]
            lo = b.offsets[tl_id]
            seen = set()
            for k, tr in enumerate(tracks):
                assert tr["track"] == k
                h = res.hit_index[tr["hit_offset"]:tr["hit_offset"] + tr["n_hits"]]
                assert 3 <= len(h) <= TW.max_track_hits
                assert not (set(h.tolist()) & seen)
                seen |= set(h.tolist())
                vv = b.vane[lo + h].astype(int)
                assert np.all((np.diff(vv) % 40) == 1)               # consecutive vanes
                tt = b.t[lo + h]
                assert np.all(np.abs(np.diff(tt)) <= TW.gate_t)       # time gate between neighbours
                w0, w1 = tr["window"], tr["last_window"]
                assert tt.min() >= np.float32(w0 * TW.step_ns) and tt.max() < np.float32(w1 * TW.step_ns) + 10
                assert tr["vane_first"] == vv[0] and tr["vane_last"] == vv[-1]
            # creation order: windows non-decreasing
            assert np.all(np.diff(tracks["window"]) >= 0)
        # offsets of the output cover the hit list exactly
        assert np.array_equal(np.concatenate([[0], np.cumsum(res.tracks["n_hits"])[:-1]]), res.tracks["hit_offset"])


def test_degenerate_inputs():
    e = np.zeros(0, np.float32)
    res = oracle_tw_find_batch(CFG, TW, np.array([0, 0]), e, e, np.zeros(0, np.int16), e, 3)
    assert len(res.tracks) == 0
    r, z, v, t = curve(10)
    assert len(run(r, z, v, t, n_windows=0).tracks) == 0
    for bad in ("unsorted", "negative", "nan"):
        tt = t.astype(np.float32).copy()
        if bad == "unsorted":
            tt[3], tt[4] = tt[4], tt[3]
        elif bad == "negative":
            tt[0] = -1.0
        else:
            tt[5] = np.nan
        with pytest.raises(OracleError) as ei:
            oracle_tw_find_batch(CFG, TW, np.array([0, 10]), r, z, v, tt, 2)
        assert ei.value.status == -6
