"""The allocation-free finder entry point (hough_find_noalloc) through the C
ABI: its output equals hough_find's byte for byte (and the oracle's), on
calls in a row whose inputs shrink, on one-event calls and on an event that
overflows its smaller large-event peak lists; oversized calls are refused
before anything is enqueued."""
import numpy as np
import pytest

from oracle import oracle_find_batch
from paper_2511_02742_amd import eventgen
from test_gpu_parity import _ocfg, assert_same, finder

pytestmark = pytest.mark.gpu


def _run(f, b, noalloc):
    import torch
    dev = torch.device("cuda", 0)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.vane).to(dev)
    o = torch.from_numpy(b.offsets).to(dev)
    out = f.alloc_outputs(b.n_events, b.n_hits)
    f.find(z, v, o, out=out, noalloc=noalloc)
    torch.cuda.synchronize(dev)
    return out.to_host()


def _same_bytes(a, b, what, all_counts=True):
    ca, ha, ia = a
    cb, hb, ib = b
    assert ia["status"] == 0 and ib["status"] == 0, (what, ia, ib)
    assert np.array_equal(ca.view(np.uint8), cb.view(np.uint8)), what
    assert np.array_equal(ha, hb), what
    if all_counts:
        assert ia == ib, (what, ia, ib)
    else:
        for k in ("candidates", "hits", "status", "detail", "iters", "max_iters"):
            assert ia[k] == ib[k], (what, k, ia[k], ib[k])


def test_noalloc_equals_find_on_shrinking_calls(gpu_available):
    f = finder()
    first = eventgen.pileup_batch(600, seed0=21000)       # more events than resident workgroups
    second = eventgen.poisson_batch(40, seed0=21500)      # smaller, after it
    for b, what in ((first, "first call, 600 pileup-50 events"), (second, "second call, 40 events")):
        got = _run(f, b, True)
        ref = _run(f, b, False)
        _same_bytes(got, ref, what)
        assert_same(got, oracle_find_batch(_ocfg(f.config), b.offsets, b.z, b.vane), what)
    assert _run(f, first, True)[2]["ordered"] == 1


def test_noalloc_one_event_and_peak_list_overflow(gpu_available):
    f = finder()
    one = eventgen.make_batch([eventgen.pileup_event(21900)])
    _same_bytes(_run(f, one, True), _run(f, one, False), "one event")
    # pileup 150: thousands of window peaks, beyond the 4096-entry slot lists
    # of the allocation-free form (tiled sweep there), the same candidates
    big = eventgen.make_batch([eventgen.pileup_event(22000 + i, n_tracks=150) for i in range(3)])
    got, ref = _run(f, big, True), _run(f, big, False)
    _same_bytes(got, ref, "pileup 150", all_counts=False)
    assert_same(got, oracle_find_batch(_ocfg(f.config), big.offsets, big.z, big.vane), "pileup 150")


def test_noalloc_refuses_calls_beyond_its_scratch(gpu_available):
    import torch
    from paper_2511_02742_amd.hough import HOUGH_ERR_CAPACITY, HoughError
    f = finder()
    dev = torch.device("cuda", 0)
    n_ev, per = 24, 125000                        # 3 M hits: more than the 64 MiB scratch holds
    z = torch.zeros(n_ev * per, dtype=torch.float32, device=dev)
    v = torch.zeros(n_ev * per, dtype=torch.int16, device=dev)
    o = torch.arange(0, n_ev * per + 1, per, dtype=torch.int64, device=dev)
    out = f.alloc_outputs(n_ev, n_ev * per)
    out.counts.fill_(-7)
    with pytest.raises(HoughError) as ei:
        f.find(z, v, o, out=out, noalloc=True)
    assert ei.value.status == HOUGH_ERR_CAPACITY
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize(dev)
    assert int(out.counts[0]) == -7               # nothing was enqueued
    small = eventgen.poisson_batch(8, seed0=22100)
    _same_bytes(_run(f, small, True), _run(f, small, False), "after a refusal")
