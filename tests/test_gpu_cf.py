"""Parity of the coarse-to-fine finder (peak_mode 2: an 18 x 100 coarse
histogram, then the 10 x 10 fine block of its best bin, on the paper's
180 x 1000 grid) with the oracle's coarse-to-fine mode, through the C ABI.

Exact comparison: candidates, ordered hit lists, the Eq. (4) evaluation and
iteration counts, the debug histogram after k iterations. Inputs come from
the seeded generator only."""
import numpy as np
import pytest

from oracle import oracle_acc_after, oracle_find, oracle_find_batch
from paper_2511_02742_amd import eventgen
from test_gpu_parity import FIELDS, _ocfg, assert_same, finder, full_size_reference, order_edge_events

pytestmark = pytest.mark.gpu

PAPER = dict(n_theta=180, n_rho=1000, peak_mode=2)


def check(batch, what="", **kw):
    cfg = dict(PAPER)
    cfg.update(kw)
    f = finder(**cfg)
    got = f.find_host(batch.z, batch.vane, batch.offsets)
    want = oracle_find_batch(_ocfg(f.config), batch.offsets, batch.z, batch.vane)
    assert_same(got, want, what)
    info = got[2]
    assert info["evals"] == expected_evals(f.config, batch.offsets, want.cand), (what, info["evals"])
    assert info["votes"] == info["evals"]          # every evaluation is an LDS vote here
    assert info["max_iters"] == want.n_iters, what
    # one candidate per iteration: no iteration ends without one
    assert info["iters"] == info["candidates"], what
    return got, want


def expected_evals(cfg, offsets, cand):
    """Eq. (4) evaluations of the coarse-to-fine kernel, from the oracle's
    candidates: the coarse histogram of every hit once, the fine block of the
    alive hits in every iteration, and the coarse votes of each candidate's
    hits when they are removed (unless the iteration cap ends the loop)."""
    ct = cfg.coarse_theta or 10
    c_rows = cfg.n_theta // ct
    T = cfg.min_votes
    total = 0
    for e in range(len(offsets) - 1):
        n = int(offsets[e + 1] - offsets[e])
        hits = [int(c["n_hits"]) for c in cand[cand["event"] == e]]
        alive, it = n, 0
        while cfg.max_iters == 0 or it < cfg.max_iters:
            if alive < T:
                break
            if it == 0:
                total += n * c_rows
            total += alive * ct
            if it == len(hits):
                break                   # the fine maximum fell below T
            if cfg.max_iters == 0 or it + 1 < cfg.max_iters:
                total += hits[it] * c_rows
            alive -= hits[it]
            it += 1
    return total


@pytest.mark.parametrize("pileup", [1, 10, 25, 50, 100, 150])
def test_pileup_levels(gpu_available, pileup):
    b = eventgen.pileup_batch(12, n_tracks=pileup, seed0=7000 + pileup)
    got, want = check(b, "pileup %d" % pileup)
    if pileup >= 10:
        assert len(want.cand) > 0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_single_event(gpu_available, seed):
    # one event: the kernel writes the caller's outputs and counts itself
    check(eventgen.make_batch([eventgen.pileup_event(seed)]), "single %d" % seed)


@pytest.mark.parametrize("kw", [{"assoc_window": 1}, {"assoc_window": 3}, {"min_votes": 4}, {"min_votes": 9},
                                {"max_iters": 1}, {"max_iters": 3}, {"phi_unit": 1},
                                {"wg_threads": 512}, {"wg_threads": 1024},
                                {"coarse_theta": 5, "coarse_rho": 20}, {"coarse_theta": 18, "coarse_rho": 50},
                                {"coarse_theta": 1, "coarse_rho": 1000}, {"coarse_theta": 180, "coarse_rho": 1},
                                {"n_theta": 360, "n_rho": 2000, "coarse_theta": 20, "coarse_rho": 20}])
def test_config_variants(gpu_available, kw):
    b = eventgen.pileup_batch(10, n_tracks=40, seed0=7300)
    check(b, str(kw), **kw)


def test_uneven_batch(gpu_available):
    check(eventgen.poisson_batch(256, seed0=7400), "poisson batch")


def test_large_events_read_hits_from_device_memory(gpu_available):
    # beyond 1024 hits an event keeps its hits in device memory
    evs = [eventgen.pileup_event(7500 + s, n_tracks=nt) for s, nt in enumerate((300, 600, 150, 1200))]
    b = eventgen.make_batch(evs)
    assert max(e.n_hits for e in evs) > 1024 and min(e.n_hits for e in evs) <= 1024
    got, want = check(b, "large")
    assert got[2]["large"] > 0
    for e in evs[:2]:
        got1, _ = check(eventgen.make_batch([e]), "large alone")
        assert got1[2]["large"] == got1[2]["passes"]


def test_largest_event(gpu_available):
    # the largest event a call accepts, several association segments
    rng = np.random.default_rng(7600)
    n = 131072
    e = eventgen.pileup_event(7601, n_tracks=300)
    reps = n // e.n_hits + 1
    z = np.concatenate([e.z + np.float32(0.25 * i) for i in range(reps)])[:n].astype(np.float32)
    v = np.concatenate([e.vane] * reps)[:n]
    perm = rng.permutation(n)
    z, v = z[perm], v[perm]
    f = finder(max_iters=3, **PAPER)
    cand, hits, info = f.find_host(z, v, np.array([0, n], np.int64))
    want = oracle_find(_ocfg(f.config), z, v)
    assert info["status"] == 0 and info["candidates"] == len(want.cand) > 0
    for fld in FIELDS:
        assert np.array_equal(cand[fld], want.cand[fld]), fld
    assert np.array_equal(hits, want.hit_index)
    assert info["evals"] == expected_evals(f.config, np.array([0, n]), want.cand)


def test_edge_events(gpu_available):
    evs = [eventgen.make_event(1, 5, noise_frac=0.0), eventgen.make_event(1, 0, noise_frac=0.0)]
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
    far = eventgen.pileup_event(14)
    far.z = np.full_like(far.z, np.float32(9.0e5))                    # every vote outside the rho range
    evs.append(far)
    exact = eventgen.pileup_event(15, n_tracks=1)
    exact.z = exact.z[:0]
    exact.vane = exact.vane[:0]
    exact.r = exact.r[:0]
    exact.track = exact.track[:0]
    evs.append(exact)                                                 # empty
    evs.append(eventgen.pileup_event(16, n_tracks=5))
    b = eventgen.make_batch(evs)
    check(b, "edges")
    for e in evs:
        check(eventgen.make_batch([e]), "edge alone")


def test_empty_batch(gpu_available):
    f = finder(**PAPER)
    b = eventgen.make_batch([])
    cand, hits, info = f.find_host(b.z, b.vane, b.offsets)
    assert info["status"] == 0 and info["candidates"] == 0 and info["hits"] == 0


@pytest.mark.parametrize("iters", [0, 1, 2, 4])
def test_debug_accumulator(gpu_available, iters):
    f = finder(**PAPER)
    e = eventgen.pileup_event(17, n_tracks=30)
    acc, info = f.debug_accumulator(e.z, e.vane, iters)
    assert info["status"] == 0
    assert np.array_equal(acc, oracle_acc_after(_ocfg(f.config), e.z, e.vane, iters))


def test_invalid_hits_reported(gpu_available):
    f = finder(**PAPER)
    b = eventgen.pileup_batch(4, seed0=7700)
    vane = b.vane.copy()
    vane[b.offsets[2] + 5] = 40
    cand, hits, info = f.find_host(b.z, vane, b.offsets)
    assert info["status"] == -6 and info["detail"] == b.offsets[2] + 5 and info["candidates"] == 0
    one = eventgen.make_batch([b.events[1]])
    z = one.z.copy()
    z[3] = np.inf
    cand, hits, info = f.find_host(z, one.vane, one.offsets)
    assert info["status"] == -6 and info["detail"] == 3
    check(b, "after error")


def test_full_size_batch(gpu_available):
    # 4096 pileup-50 events in one launch, run longest first: every event
    # byte-equal to the oracle, and the evaluation count derived from it
    b = eventgen.pileup_batch(4096)
    f = finder(**PAPER)
    got = f.find_host(b.z, b.vane, b.offsets)
    want = full_size_reference(_ocfg(f.config), b)
    assert_same(got, want, "coarse-to-fine full-size batch")
    assert got[2]["ordered"] == 1, got[2]
    assert got[2]["evals"] == expected_evals(f.config, b.offsets, want.cand)


def test_longest_first_order_edge_sizes(gpu_available):
    # more events than resident coarse-to-fine workgroups (256 threads, about
    # 17 KB of LDS: 8 per CU, 2048 on the device): ordered, every event once
    evs = order_edge_events(2600, seed0=13000)
    got, want = check(eventgen.make_batch(evs), "cf order edges")
    assert got[2]["ordered"] == 1, got[2]
    got, _ = check(eventgen.make_batch(evs[:1500]), "cf order edges, 1500 events")
    assert got[2]["ordered"] == 0, got[2]


def test_graph_replays_match_oracle(gpu_available):
    # captured launch, replayed with eager work and synchronisations between
    # the replays; every replay against the oracle
    import torch
    f = finder(**PAPER)
    b = eventgen.poisson_batch(64, seed0=7800)
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    want = oracle_find_batch(_ocfg(f.config), b.offsets, b.z, b.vane)
    other = eventgen.pileup_batch(3, seed0=7900)
    g = f.capture(z, v, o)
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize(dev)
        assert_same(out.to_host(), want, "replay %d" % rep)
        check(other, "eager between replays")
    g.close()
