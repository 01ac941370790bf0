"""Input generator: reproducible, on the strip grid, inside the detector."""
import numpy as np

from paper_2511_02742_amd import eventgen as g


def test_seed_reproducible():
    a = g.pileup_event(17)
    b = g.pileup_event(17)
    assert np.array_equal(a.z, b.z) and np.array_equal(a.vane, b.vane) and np.array_equal(a.r, b.r)
    c = g.pileup_event(18)
    assert not (a.n_hits == c.n_hits and np.array_equal(a.z, c.z))


def test_hits_on_strip_grid_and_in_range():
    e = g.pileup_event(3)
    assert e.z.dtype == np.float32 and e.vane.dtype == np.int16 and e.r.dtype == np.float32
    assert np.all((e.vane >= 0) & (e.vane < 40))
    assert np.all((e.r >= 90.0) & (e.r <= 290.1)) and np.all(np.abs(e.z) <= 200.0)
    iz = (e.z.astype(np.float64) + 200.0) / 0.19 - 0.5
    ir = (e.r.astype(np.float64) - 90.0) / 0.19 - 0.5
    assert np.allclose(iz, np.round(iz), atol=1e-3) and np.allclose(ir, np.round(ir), atol=1e-3)


def test_noise_fraction():
    e = g.pileup_event(5)
    n_sig = int((e.track >= 0).sum())
    assert int((e.track < 0).sum()) == int(np.floor(0.01 * n_sig + 0.5))
    t = g.tiny_event(0)
    assert (t.track >= 0).all() and t.n_tracks == 5


def test_batch_offsets():
    b = g.poisson_batch(20, seed0=5)
    assert b.offsets[0] == 0 and b.offsets[-1] == b.n_hits == b.z.shape[0]
    assert np.all(np.diff(b.offsets) >= 0)
    for i, e in enumerate(b.events):
        assert np.array_equal(b.z[b.offsets[i]:b.offsets[i + 1]], e.z)
    h = g.hit_histogram(b)
    assert h["n_events"] == 20 and h["hits_min"] <= h["hits_mean"] <= h["hits_max"]


def test_tracks_are_helices_near_lines_in_phi_z():
    # a track's hits on one turn lie close to a line in (vane azimuth, z)
    e = g.make_event(101, 30, noise_frac=0.0)
    for t in range(30):
        m = e.track == t
        if m.sum() < 8:
            continue
        assert np.ptp(e.z[m]) <= 400.0
