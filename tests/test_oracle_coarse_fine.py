"""Pins of the oracle's coarse-to-fine mode (peak_mode 2; the paper's 18 x 100
coarse histogram refined by a 10 x 10 fine one inside the most likely coarse
region, Sec. 6 and Fig. 4). The coarse and fine histograms are checked
against the oracle's plain histogram fill on the coarse grid and on the full
grid, a different code path that is the definition of both."""
import math

import numpy as np
import pytest

from oracle import OracleConfig, oracle_fill, oracle_find
from oracle.oracle import OracleError
from paper_2511_02742_amd import eventgen


def _key(count, flat):
    return (int(count) << 32) | (0xFFFFFFFF - int(flat))


def _cfg(**kw):
    base = dict(n_theta=180, n_rho=1000, min_votes=6, peak_mode=2, coarse_theta=10, coarse_rho=10)
    base.update(kw)
    return OracleConfig(**base)


def _first_peak_by_definition(z, vane, c):
    """The coarse-to-fine peak from two plain fills: the coarse histogram on the
    coarse grid, its largest key, then the full histogram's largest key inside
    that bin's block."""
    coarse = OracleConfig(n_theta=c.n_theta // c.coarse_theta, n_rho=c.n_rho // c.coarse_rho,
                          rho_min=c.rho_min, rho_max=c.rho_max)
    acc_c, _ = oracle_fill(coarse, z, vane)
    keys = [_key(acc_c.flat[b], b) for b in range(acc_c.size)]
    b = int(np.argmax(keys))
    J, K = divmod(b, coarse.n_rho)
    full = OracleConfig(n_theta=c.n_theta, n_rho=c.n_rho, rho_min=c.rho_min, rho_max=c.rho_max)
    acc, _ = oracle_fill(full, z, vane)
    best = 0
    for j in range(J * c.coarse_theta, (J + 1) * c.coarse_theta):
        for k in range(K * c.coarse_rho, (K + 1) * c.coarse_rho):
            best = max(best, _key(acc[j, k], j * c.n_rho + k))
    flat = 0xFFFFFFFF - (best & 0xFFFFFFFF)
    return divmod(flat, c.n_rho) + (best >> 32,), acc


@pytest.mark.parametrize("seed", [0, 3, 7, 11])
def test_first_peak_is_the_fine_maximum_of_the_best_coarse_block(seed):
    ev = eventgen.pileup_event(seed, n_tracks=25)
    c = _cfg(max_iters=1)
    r = oracle_find(c, ev.z, ev.vane)
    (j, k, cnt), acc = _first_peak_by_definition(ev.z, ev.vane, c)
    assert len(r.cand) == (1 if cnt >= 6 else 0)
    if len(r.cand):
        cd = r.cand[0]
        assert (cd["theta_bin"], cd["rho_bin"], cd["peak_votes"]) == (j, k, cnt)
        # with a = 0 the seed is exactly the hits voting into that fine bin
        assert cd["n_hits"] == acc[j, k]


def _line(jstar, kstar):
    th = (jstar + 0.5) * math.pi / 180
    rho = -500.0 + (kstar + 0.5) * 1.0
    vanes, zs = [], []
    for v in range(40):
        phi = 9.0 * v
        z = (rho - phi * math.cos(th)) / math.sin(th)
        if abs(z) <= 200.0:
            vanes.append(v)
            zs.append(z)
    return zs, vanes


def test_single_line_aligned_with_its_coarse_cell():
    # hits on an exact line through fine bin (64, 415): 0.5 degrees from the
    # coarse theta sample of its coarse cell (6, 41) and in the middle of that
    # cell's rho range, so at coarse resolution all hits stay in the cell and
    # the fine block holds the line's bin: one candidate with every hit
    c = _cfg()
    zs, vanes = _line(64, 415)
    m = len(vanes)
    assert m >= 8
    r = oracle_find(c, zs, vanes)
    assert len(r.cand) == 1 and r.cand[0]["n_hits"] == m and r.cand[0]["peak_votes"] == m
    full, _ = oracle_fill(OracleConfig(n_theta=180, n_rho=1000), zs, vanes)
    assert full.max() == m and full[r.cand[0]["theta_bin"], r.cand[0]["rho_bin"]] == m


def test_single_line_split_by_the_coarse_grid():
    # the same line through fine bin (63, 412): 1.5 degrees from the coarse
    # sample its hits spread over several coarse rho cells, the largest one's
    # block misses the line's bin, and only parts of the line come out (the
    # rest stays below the threshold), while the full-grid argmax takes the
    # whole line in one candidate
    zs, vanes = _line(63, 412)
    m = len(vanes)
    full, _ = oracle_fill(OracleConfig(n_theta=180, n_rho=1000), zs, vanes)
    assert full[63, 412] == m
    r = oracle_find(_cfg(), zs, vanes)
    assert len(r.cand) >= 1
    assert all(6 <= c["peak_votes"] < m for c in r.cand)
    got = np.concatenate([r.hit_index[c["hit_offset"]:c["hit_offset"] + c["n_hits"]] for c in r.cand])
    assert len(np.unique(got)) == len(got) < m
    a = oracle_find(OracleConfig(n_theta=180, n_rho=1000), zs, vanes)
    assert len(a.cand) == 1 and a.cand[0]["n_hits"] == m


def test_loop_invariants_pileup():
    # an event of 25 positrons on which the loop runs six times
    ev = eventgen.pileup_event(25, n_tracks=25)
    c = _cfg()
    r = oracle_find(c, ev.z, ev.vane)
    assert len(r.cand) >= 3
    seen = set()
    for i, cd in enumerate(r.cand):
        hs = r.hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]
        assert cd["iter"] == i                     # one peak per iteration
        assert cd["n_hits"] >= 6 and cd["n_hits"] == cd["peak_votes"]
        assert np.all(np.diff(hs) > 0) and not (seen & set(hs.tolist()))
        seen |= set(hs.tolist())


def test_differs_from_the_full_argmax_on_pileup():
    # the two are not the same search: the full histogram's maximum need not
    # lie in the block of the largest coarse bin. Measured, not assumed.
    differ = 0
    n = 12
    for s in range(n):
        ev = eventgen.pileup_event(100 + s, n_tracks=50)
        a = oracle_find(OracleConfig(n_theta=180, n_rho=1000, peak_mode=0, max_iters=1), ev.z, ev.vane)
        b = oracle_find(_cfg(max_iters=1), ev.z, ev.vane)
        ka = (a.cand[0]["theta_bin"], a.cand[0]["rho_bin"]) if len(a.cand) else None
        kb = (b.cand[0]["theta_bin"], b.cand[0]["rho_bin"]) if len(b.cand) else None
        differ += ka != kb
        if len(b.cand) and len(a.cand):
            assert b.cand[0]["peak_votes"] <= a.cand[0]["peak_votes"]
    assert 0 < differ < n


def test_coarse_factors_must_divide_the_grid():
    with pytest.raises(OracleError):
        oracle_find(_cfg(coarse_theta=7), [0.0], [0])
    with pytest.raises(OracleError):
        oracle_find(_cfg(coarse_rho=0), [0.0], [0])
